"""Summaries of rocprofv3 result databases (SQLite, as written by rocprofv3 on ROCm 7).

    python -m paper_1410_3677_amd.rocprof_summary trace RESULTS.db [--match k_tmpl] [--last N]
        per-kernel dispatch statistics (calls, total, average, min, max duration) as markdown;
        --last N: only the last N dispatches of each kernel (for instance the timed steps
        of a run that starts with warm-up steps)

    python -m paper_1410_3677_amd.rocprof_summary counters RESULTS.db [--match k_tmpl]
        average of every collected counter per dispatch of each kernel (summed over
        hardware instances) as markdown

    python -m paper_1410_3677_amd.rocprof_summary traffic FETCH.db WRITE.db --copy-bytes B \
            --copy-match MulFunctor --templates-per-launch T [--kernel KEY=SUBSTRING ...] [--json OUT]
        average FETCH_SIZE / WRITE_SIZE per dispatch of each kernel, scaled by what the
        same counters read for a plain copy kernel that moves a known number of bytes;
        --kernel names the template kernels (default: template_a = k_tmpl_a,
        template_b = k_tmpl_b; the first matching entry wins)
"""
from __future__ import annotations

import argparse
import collections
import json
import sqlite3
import sys


def _short(name: str) -> str:
    n = name.replace("(anonymous namespace)::", "").split("(")[0]
    return n.replace("void ", "").replace("fstat::", "")


def trace(db: str, match: str = "", last: int = 0):
    c = sqlite3.connect(db)
    if last > 0:
        per = collections.defaultdict(list)
        for name, start, dur in c.execute("select name, start, duration from kernels order by start"):
            per[name].append(dur)
        rows = []
        for name, d in per.items():
            d = d[-last:]
            rows.append((name, len(d), sum(d), sum(d) / len(d), min(d), max(d)))
        rows.sort(key=lambda r: -r[2])
    else:
        rows = c.execute("select name, count(*), sum(duration), avg(duration), min(duration), max(duration) "
                         "from kernels group by name order by sum(duration) desc").fetchall()
    out = ["| kernel | calls | total (us) | avg (us) | min (us) | max (us) |", "|---|---|---|---|---|---|"]
    for name, n, tot, avg, mn, mx in rows:
        if match and match not in name:
            continue
        out.append(f"| `{_short(name)}` | {n} | {tot / 1e3:.1f} | {avg / 1e3:.2f} | {mn / 1e3:.2f} | {mx / 1e3:.2f} |")
    return "\n".join(out)


def counter_means(db: str, counter: str):
    """Average value of `counter` per dispatch, by kernel name (summed over hardware instances)."""
    c = sqlite3.connect(db)
    rows = c.execute("select dispatch_id, kernel_name, sum(value) from counters_collection "
                     "where counter_name = ? group by dispatch_id", (counter,)).fetchall()
    acc = collections.defaultdict(list)
    for _, k, v in rows:
        acc[k].append(v)
    return {k: (sum(v) / len(v), len(v)) for k, v in acc.items()}


def counters(db: str, match: str = ""):
    """Per-kernel averages of every counter in a --pmc results database."""
    c = sqlite3.connect(db)
    names = [r[0] for r in c.execute("select distinct counter_name from counters_collection order by counter_name")]
    cols = {n: counter_means(db, n) for n in names}
    kernels = sorted({k for m in cols.values() for k in m})
    out = ["| kernel | dispatches | " + " | ".join(names) + " |", "|---|---|" + "---|" * len(names)]
    for k in kernels:
        if match and match not in k:
            continue
        n = max(cols[nm].get(k, (0.0, 0))[1] for nm in names)
        vals = " | ".join(f"{cols[nm].get(k, (0.0, 0))[0]:.6g}" for nm in names)
        out.append(f"| `{_short(k)}` | {n} | {vals} |")
    return "\n".join(out)


def traffic(fetch_db: str, write_db: str, copy_bytes: int, copy_match: str, tpl: int, kernel_keys=None):
    keys = kernel_keys or [("template_a", "k_tmpl_a"), ("template_b", "k_tmpl_b")]
    fetch = counter_means(fetch_db, "FETCH_SIZE")
    write = counter_means(write_db, "WRITE_SIZE")
    copy_f = [v for k, (v, n) in fetch.items() if copy_match in k]
    copy_w = [v for k, (v, n) in write.items() if copy_match in k]
    if not copy_f or not copy_w:
        raise SystemExit(f"no dispatch matching {copy_match!r} for the copy calibration")
    # counters are in KiB; scale = true bytes / (counter KiB * 1024)
    sf = copy_bytes / (max(copy_f) * 1024.0)
    sw = copy_bytes / (max(copy_w) * 1024.0)
    res = {"copy_bytes": copy_bytes, "fetch_scale": sf, "write_scale": sw, "kernels": {}}
    for k in sorted(set(fetch) | set(write)):
        if "k_tmpl" not in k and "k_spline" not in k and "k_fft" not in k and "k_sky" not in k:
            continue
        f_kib = fetch.get(k, (0.0, 0))[0]
        w_kib = write.get(k, (0.0, 0))[0]
        short = _short(k)
        key = next((name for name, sub in keys if sub in short), short)
        res["kernels"][key] = {"kernel": short, "fetch_kib_raw": f_kib, "write_kib_raw": w_kib,
                               "fetch_bytes": f_kib * 1024 * sf, "write_bytes": w_kib * 1024 * sw,
                               "bytes_per_launch": f_kib * 1024 * sf + w_kib * 1024 * sw,
                               "templates_per_launch": tpl if key.startswith("template") else None}
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("--match", default="")
    t.add_argument("--last", type=int, default=0)
    cn = sub.add_parser("counters")
    cn.add_argument("db")
    cn.add_argument("--match", default="")
    f = sub.add_parser("traffic")
    f.add_argument("fetch_db")
    f.add_argument("write_db")
    f.add_argument("--copy-bytes", type=int, required=True)
    f.add_argument("--copy-match", default="MulFunctor")
    f.add_argument("--templates-per-launch", type=int, required=True)
    f.add_argument("--kernel", action="append", default=[], metavar="KEY=SUBSTRING")
    f.add_argument("--json", default="")
    f.add_argument("--source-sha256", default="")
    f.add_argument("--variants", type=int, default=-1,
                   help="kernel variants of the profiled plan: pass_a_variant + 2 pass_b_variant")
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        print(trace(a.db, a.match, a.last))
    elif a.cmd == "counters":
        print(counters(a.db, a.match))
    else:
        keys = [tuple(x.split("=", 1)) for x in a.kernel] or None
        res = traffic(a.fetch_db, a.write_db, a.copy_bytes, a.copy_match, a.templates_per_launch, keys)
        if a.source_sha256:
            res["source_sha256"] = a.source_sha256
        if a.variants >= 0:
            res["variants"] = a.variants
        text = json.dumps(res, indent=1)
        if a.json:
            with open(a.json, "w") as fh:
                fh.write(text + "\n")
        print(text)


if __name__ == "__main__":
    main(sys.argv[1:])
