"""Short text summaries of rocprofv3 result databases, for the files under profiles/.

    python -m paper_2305_14306_amd.profile_report stats RESULTS_DB OUT.txt --command "..."
    python -m paper_2305_14306_amd.profile_report pmc FETCH_DB WRITE_DB OUT.txt --kernel k_search \
        --command-fetch "..." --command-write "..."
    python -m paper_2305_14306_amd.profile_report counters RESULTS_DB OUT.txt --command "..."

`stats` lists every kernel of a --kernel-trace --stats run (calls, total, average).
`counters` lists, per kernel, the average per dispatch of every counter of one --pmc run.
`pmc` turns two counter runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch) into HBM
bytes per launch of one kernel. Each counter is scaled by the factor that makes it read
the known traffic of a plain elementwise kernel of the same runs (bench.py
--copy-calib: neg over 64 Mi float32, 256 MiB read and 256 MiB written). The summary
records a digest of the kernel sources so that bench.py can tell whether the counters
still describe the code it runs.
"""
from __future__ import annotations

import argparse
import hashlib
import os
import re
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = (os.path.join(ROOT, "paper_2305_14306_amd", "csrc", "hav.hip"),
           os.path.join(ROOT, "paper_2305_14306_amd", "csrc", "hav_device.hpp"))
CALIB_KIB = 256 * 1024  # the calibration kernel reads and writes 256 MiB


def _code_only(text: str) -> str:
    """The source with // comments and blank lines removed (comments do not change
    what the counters measured)."""
    out = []
    for line in text.splitlines():
        code = line.split("//", 1)[0].rstrip() if "//" in line and '"' not in line else line.rstrip()
        if code:
            out.append(code)
    return "\n".join(out)


def source_digest() -> str:
    h = hashlib.sha256()
    for f in SOURCES:
        with open(f, encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    m = re.search(r"\b(k_\w+)\s*[<(]", name)
    if m:
        # the batched path's instantiations (template argument Many) are named apart
        rest, tmpl, depth = name[m.end(1):].lstrip(), "", 0
        for ch in rest if rest.startswith("<") else "":
            depth += (ch == "<") - (ch == ">")
            tmpl += ch
            if depth == 0:
                break
        return m.group(1) + (" (batch)" if re.search(r"\bMany\b", tmpl) else "")
    if "neg_kernel" in name:
        return "calib_neg (torch elementwise)"
    if "FillFunctor" in name:
        return "torch fill"
    return name.split("(")[0][:48]


def stats(db: str) -> list:
    """(kernel, calls, total us, average us, percent) from the top_kernels view, whose
    durations are in microseconds."""
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels")
    return [(short_name(n), int(c), float(t), float(a), float(p)) for n, c, t, a, p in rows]


def counter_per_dispatch(db: str, counter: str) -> dict:
    con = sqlite3.connect(db)
    out: dict = {}
    q = "select kernel_name, value from counters_collection where counter_name = ?"
    for name, val in con.execute(q, (counter,)):
        out.setdefault(short_name(name), []).append(float(val))
    return out


def write_stats(args) -> None:
    rows = stats(args.db)
    lines = [f"# rocprofv3 kernel summary", f"# command: {args.command}",
             f"# {'kernel':30s} {'calls':>6s} {'total_us':>11s} {'avg_us':>9s} {'pct':>6s}"]
    for n, c, t, a, p in rows:
        lines.append(f"{n:32s} {c:6d} {t:11.1f} {a:9.2f} {p:6.2f}")
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def write_pmc(args) -> None:
    fetch = counter_per_dispatch(args.fetch_db, "FETCH_SIZE")
    write = counter_per_dispatch(args.write_db, "WRITE_SIZE")
    calib = "calib_neg (torch elementwise)"
    f_cal, w_cal = fetch[calib][-1], write[calib][-1]
    ff, fw = CALIB_KIB / f_cal, CALIB_KIB / w_cal
    fk = sum(fetch[args.kernel]) / len(fetch[args.kernel])
    wk = sum(write[args.kernel]) / len(write[args.kernel])
    hbm = (fk * ff + wk * fw) * 1024.0
    lines = [
        f"# HBM traffic of {args.kernel} from rocprofv3 counters (KiB per dispatch)",
        f"# fetch run: {args.command_fetch}",
        f"# write run: {args.command_write}",
        f"# calibration: elementwise neg over 64 Mi float32 reads {CALIB_KIB} KiB and writes "
        f"{CALIB_KIB} KiB; counters read {f_cal:.1f} and {w_cal:.1f}",
        f"kernel = {args.kernel}",
        f"dispatches = {len(fetch[args.kernel])}",
        f"fetch_kib_per_dispatch = {fk:.1f}",
        f"write_kib_per_dispatch = {wk:.1f}",
        f"fetch_scale = {ff:.4f}",
        f"write_scale = {fw:.4f}",
        f"hbm_bytes_per_launch = {hbm:.0f}",
        f"source_digest = {source_digest()}",
        "# all kernels, average KiB per dispatch (fetch, write), unscaled:",
    ]
    for k in sorted(set(fetch) | set(write)):
        fv = fetch.get(k, [0.0])
        wv = write.get(k, [0.0])
        lines.append(f"#   {k:32s} {sum(fv) / len(fv):12.1f} {sum(wv) / len(wv):12.1f}")
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def write_counters(args) -> None:
    con = sqlite3.connect(args.db)
    names = sorted({r[0] for r in con.execute("select distinct counter_name from counters_collection")})
    per = {c: counter_per_dispatch(args.db, c) for c in names}
    kernels = sorted({k for c in names for k in per[c]})
    lines = [f"# rocprofv3 counters, average per dispatch", f"# command: {args.command}",
             f"# {'kernel':30s} {'dispatches':>10s} " + " ".join(f"{c:>32s}" for c in names)]
    for k in kernels:
        n = len(per[names[0]].get(k, []))
        vals = []
        for c in names:
            v = per[c].get(k, [0.0])
            vals.append(sum(v) / len(v))
        lines.append(f"{k:32s} {n:10d} " + " ".join(f"{v:32.0f}" for v in vals))
    with open(args.out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("out")
    s.add_argument("--command", required=True)
    p = sub.add_parser("pmc")
    p.add_argument("fetch_db")
    p.add_argument("write_db")
    p.add_argument("out")
    p.add_argument("--kernel", default="k_search")
    p.add_argument("--command-fetch", required=True)
    p.add_argument("--command-write", required=True)
    c = sub.add_parser("counters")
    c.add_argument("db")
    c.add_argument("out")
    c.add_argument("--command", required=True)
    args = ap.parse_args(argv)
    if args.what == "stats":
        write_stats(args)
    elif args.what == "counters":
        write_counters(args)
    else:
        write_pmc(args)
    return 0


if __name__ == "__main__":
    sys.exit(main())
