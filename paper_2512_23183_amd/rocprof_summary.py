"""Short text summaries of rocprofv3 SQLite results (``*_results.db``).

  python -m paper_2512_23183_amd.rocprof_summary stats DB [--match REGEX] [--last N]
      per-kernel dispatch count, total / mean / min / max duration and the
      launch shape of the last dispatch (the ``--kernel-trace --stats`` view);
      --last keeps the last N dispatches of each kernel
  python -m paper_2512_23183_amd.rocprof_summary pmc DB [--match REGEX]
      per-kernel mean of every collected counter per dispatch
  python -m paper_2512_23183_amd.rocprof_summary traffic --kernel REGEX
      --fetch DB --write DB --copy-fetch DB --copy-write DB --copy-bytes N
      HBM bytes per dispatch of a kernel from FETCH_SIZE / WRITE_SIZE, each
      scaled by what the counter reads for a plain streaming kernel that
      reads and writes N bytes

Only reads the databases; prints Markdown.
"""
from __future__ import annotations

import argparse
import collections
import re
import sqlite3
import statistics


def _kernels(db):
    con = sqlite3.connect(db)
    rows = con.execute("select name, duration, grid_x, workgroup_x, lds_size, vgpr_count, sgpr_count, "
                       "scratch_size from kernels order by start").fetchall()
    con.close()
    return rows


def _pmc(db):
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, name, counter_name, counter_value from pmc_events").fetchall()
    con.close()
    per = collections.defaultdict(dict)
    names = {}
    for did, name, cn, cv in rows:
        per[did][cn] = per[did].get(cn, 0.0) + float(cv)
        names[did] = name
    return per, names


def short(name: str) -> str:
    name = name.split("(")[0]
    return name.replace("void ", "")


def stats(db, match=None, last=0):
    groups = collections.OrderedDict()
    for name, dur, gx, wx, lds, vgpr, sgpr, scratch in _kernels(db):
        if match and not re.search(match, name):
            continue
        g = groups.setdefault(short(name), {"d": [], "shape": (gx, wx, lds, vgpr, sgpr, scratch)})
        g["d"].append(dur / 1e3)  # ns -> us
        g["shape"] = (gx, wx, lds, vgpr, sgpr, scratch)
    if last:
        # the workload of interest runs at the end of the command
        for g in groups.values():
            g["d"] = g["d"][-last:]
    out = ["| kernel | calls | total ms | avg us | min us | max us | grid | wg | LDS B | VGPR | SGPR | scratch |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for k, g in sorted(groups.items(), key=lambda kv: -sum(kv[1]["d"])):
        d = g["d"]
        gx, wx, lds, vgpr, sgpr, scratch = g["shape"]
        out.append(f"| {k} | {len(d)} | {sum(d) / 1e3:.3f} | {statistics.mean(d):.1f} | {min(d):.1f} | "
                   f"{max(d):.1f} | {gx} | {wx} | {lds} | {vgpr} | {sgpr} | {scratch} |")
    return "\n".join(out)


def by_position(db, match, last, period):
    """Durations of the last `last` dispatches matching `match`, grouped by
    their position modulo `period` (e.g. the passes of one step)."""
    d = [dur / 1e3 for name, dur, *_ in _kernels(db) if re.search(match, name)][-last:]
    out = ["| position | dispatches | avg us | min us | max us |", "|---|---|---|---|---|"]
    for p in range(period):
        x = d[p::period]
        if x:
            out.append(f"| {p} | {len(x)} | {statistics.mean(x):.1f} | {min(x):.1f} | {max(x):.1f} |")
    return "\n".join(out)


def pmc(db, match=None):
    per, names = _pmc(db)
    agg = collections.OrderedDict()
    for did in sorted(per):
        name = names[did]
        if match and not re.search(match, name):
            continue
        a = agg.setdefault(short(name), collections.defaultdict(list))
        for cn, cv in per[did].items():
            a[cn].append(cv)
    out = []
    for k, a in agg.items():
        cols = ", ".join(f"{cn} mean {statistics.mean(v):.1f} (n={len(v)})" for cn, v in sorted(a.items()))
        out.append(f"- {k}: {cols}")
    return "\n".join(out)


def counter_mean(db, counter, match):
    per, names = _pmc(db)
    vals = [v[counter] for did, v in per.items() if counter in v and re.search(match, names[did])]
    if not vals:
        raise SystemExit(f"no {counter} samples for kernels matching {match!r} in {db}")
    return statistics.mean(vals), len(vals)


def traffic(kernel, fetch_db, write_db, copy_fetch_db, copy_write_db, copy_bytes, copy_match):
    kib = 1024.0
    cf, ncf = counter_mean(copy_fetch_db, "FETCH_SIZE", copy_match)
    cw, ncw = counter_mean(copy_write_db, "WRITE_SIZE", copy_match)
    f_scale = copy_bytes / (cf * kib)
    w_scale = copy_bytes / (cw * kib)
    kf, nkf = counter_mean(fetch_db, "FETCH_SIZE", kernel)
    kw, nkw = counter_mean(write_db, "WRITE_SIZE", kernel)
    fetch_b = kf * kib * f_scale
    write_b = kw * kib * w_scale
    lines = [
        f"- plain streaming kernel ({copy_match}), {copy_bytes} B read and written per dispatch: "
        f"FETCH_SIZE {cf:.1f} KiB (n={ncf}), WRITE_SIZE {cw:.1f} KiB (n={ncw})",
        f"- scale factors (known bytes / counter bytes): fetch {f_scale:.4f}, write {w_scale:.4f}",
        f"- {kernel}: FETCH_SIZE {kf:.1f} KiB (n={nkf}), WRITE_SIZE {kw:.1f} KiB (n={nkw}) per dispatch",
        f"- scaled HBM bytes per dispatch: fetch {fetch_b:.6e}, write {write_b:.6e}",
        f"traffic_bytes_per_launch: {fetch_b + write_b:.6e}",
    ]
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("db")
    a.add_argument("--match")
    a.add_argument("--last", type=int, default=0, help="only the last N dispatches of each kernel")
    a = sub.add_parser("positions")
    a.add_argument("db")
    a.add_argument("--match", required=True)
    a.add_argument("--last", type=int, required=True)
    a.add_argument("--period", type=int, required=True)
    a = sub.add_parser("pmc")
    a.add_argument("db")
    a.add_argument("--match")
    a = sub.add_parser("traffic")
    a.add_argument("--kernel", required=True)
    a.add_argument("--fetch", required=True)
    a.add_argument("--write", required=True)
    a.add_argument("--copy-fetch", required=True)
    a.add_argument("--copy-write", required=True)
    a.add_argument("--copy-bytes", type=float, required=True)
    a.add_argument("--copy-match", default="neg|elementwise")
    args = ap.parse_args()
    if args.cmd == "stats":
        print(stats(args.db, args.match, args.last))
    elif args.cmd == "positions":
        print(by_position(args.db, args.match, args.last, args.period))
    elif args.cmd == "pmc":
        print(pmc(args.db, args.match))
    else:
        print(traffic(args.kernel, args.fetch, args.write, args.copy_fetch, args.copy_write, args.copy_bytes,
                      args.copy_match))


if __name__ == "__main__":
    main()
