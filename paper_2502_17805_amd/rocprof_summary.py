"""Summaries of rocprofv3 output for the kernels of this library.

  python -m paper_2502_17805_amd.rocprof_summary trace DIR --title T --cmd C
      per-kernel call counts and durations (from a --kernel-trace --stats run)
      plus register, LDS and scratch use, as a markdown table.
  python -m paper_2502_17805_amd.rocprof_summary traffic --fetch DIR --write DIR
      --copy-bytes B --key K --source-hash H [--kernel SUBSTR] --json OUT --cmd C
      HBM bytes per dispatch from a FETCH_SIZE run and a WRITE_SIZE run of the
      same program.  Each counter is scaled by what it reads for the plain
      device copy of B bytes in the same program (torch's elementwise copy
      kernel, which reads B and writes B bytes), so the figure is in the
      units of bytes actually moved.  Appends an entry to OUT (JSON) and
      prints a markdown summary.
  python -m paper_2502_17805_amd.rocprof_summary counters DIR [DIR ...]
      every counter of every kernel of this library in one or more --pmc
      runs, means per dispatch, as a markdown table.

Reads the SQLite databases rocprofv3 writes (tables `top_kernels`, `kernels`,
`pmc_events`).
"""
from __future__ import annotations

import argparse
import collections
import glob
import json
import os
import sqlite3
import sys


def _db(path):
    if path.endswith(".db"):
        return path
    found = sorted(glob.glob(os.path.join(path, "**", "*.db"), recursive=True))
    if not found:
        raise FileNotFoundError(f"no rocprofv3 database under {path}")
    return found[0]


def trace_table(path, title, cmd, limit=16):
    c = sqlite3.connect(_db(path))
    rows = list(c.execute("select name,total_calls,total_duration,average,percentage from top_kernels "
                          f"limit {int(limit)}"))
    res = {}
    for r in c.execute("select name, vgpr_count, accum_vgpr_count, sgpr_count, lds_size, scratch_size, "
                       "workgroup_x, grid_x from kernels group by name"):
        res[r[0]] = r[1:]
    out = [f"# {title}", "", "Command (from the repository root):", "", "```", cmd, "```", "",
           "| kernel | calls | total us | avg us | % | VGPR* | AGPR | LDS B | scratch B | wg | grid threads |",
           "|---|---|---|---|---|---|---|---|---|---|---|"]
    for n, calls, tot, avg, pct in rows:
        v = res.get(n, (None,) * 7)
        out.append(f"| `{n[:80]}` | {calls} | {tot:.0f} | {avg:.1f} | {pct:.1f} | {v[0]} | {v[1]} | "
                   f"{v[3]} | {v[4]} | {v[5]} | {v[6]} |")
    out += ["", "*VGPR as recorded by the profiler (allocation granules may differ from the compiler's count)."]
    return "\n".join(out) + "\n"


def pmc_per_kernel(path):
    """{kernel name: {counter: mean per dispatch}} (plus "duration_ns"); a
    counter reported per hardware instance is summed over instances within
    each dispatch."""
    c = sqlite3.connect(_db(path))
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for name, disp, cn, v, dur in c.execute("select name, dispatch_id, counter_name, counter_value, duration "
                                            "from pmc_events"):
        per[(name, disp)][cn] += v
        per[(name, disp)]["duration_ns"] = dur
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for (name, _), cs in per.items():
        for cn, v in cs.items():
            agg[name][cn].append(v)
    return {n: {cn: sum(v) / len(v) for cn, v in cs.items()} for n, cs in agg.items()}


def counter_table(dirs, sub="sdm::k_"):
    """Markdown table of every counter of every kernel matching `sub`, over
    one or more --pmc runs of the same program (means per dispatch)."""
    merged = collections.defaultdict(dict)
    for d in dirs:
        for n, cs in pmc_per_kernel(d).items():
            if sub in n:
                merged[n].update(cs)
    names = sorted({cn for cs in merged.values() for cn in cs if cn != "duration_ns"})
    out = ["| kernel | avg us | " + " | ".join(names) + " |", "|---" * (len(names) + 2) + "|"]
    for n, cs in merged.items():
        short = n.split("(")[0].replace("void ", "")
        out.append(f"| `{short}` | {cs.get('duration_ns', 0) / 1e3:.0f} | " +
                   " | ".join(f"{cs[c]:.4g}" if c in cs else "" for c in names) + " |")
    return "\n".join(out) + "\n"


def _pick(table, sub):
    hits = [n for n in table if sub in n]
    if not hits:
        raise KeyError(f"no kernel matching {sub!r}; have {sorted(table)[:8]}")
    return hits


def traffic(fetch_dir, write_dir, copy_bytes, kernel_sub):
    fe, wr = pmc_per_kernel(fetch_dir), pmc_per_kernel(write_dir)
    # the copy: the elementwise kernel that fetches the most (the fills that
    # initialise buffers fetch nothing)
    copy = max(_pick(fe, "elementwise_kernel"), key=lambda n: fe[n]["FETCH_SIZE"])
    cf, cw = fe[copy]["FETCH_SIZE"], wr[copy]["WRITE_SIZE"]
    kf = {n: fe[n]["FETCH_SIZE"] for n in _pick(fe, kernel_sub)}
    kw = {n: wr[n]["WRITE_SIZE"] for n in _pick(wr, kernel_sub)}
    name = max(kf, key=kf.get)
    return dict(kernel=name, fetch_kib=kf[name], write_kib=kw.get(name), copy_fetch_kib=cf, copy_write_kib=cw,
                fetch_scale=copy_bytes / cf, write_scale=copy_bytes / cw,
                bytes_per_launch=kf[name] * copy_bytes / cf + kw.get(name, 0.0) * copy_bytes / cw)


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_name", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("--title", required=True)
    t.add_argument("--cmd", required=True)
    k = sub.add_parser("counters")
    k.add_argument("dirs", nargs="+")
    k.add_argument("--kernel", default="sdm::k_")
    f = sub.add_parser("traffic")
    f.add_argument("--fetch", required=True)
    f.add_argument("--write", required=True)
    f.add_argument("--copy-bytes", type=float, required=True)
    f.add_argument("--kernel", default="k_volume")
    f.add_argument("--key", required=True)
    f.add_argument("--source-hash", required=True)
    f.add_argument("--json", required=True)
    f.add_argument("--cmd", required=True)
    a = ap.parse_args(argv)
    if a.cmd_name == "trace":
        sys.stdout.write(trace_table(a.dir, a.title, a.cmd))
        return
    if a.cmd_name == "counters":
        sys.stdout.write(counter_table(a.dirs, a.kernel))
        return
    r = traffic(a.fetch, a.write, a.copy_bytes, a.kernel)
    r["source_hash"] = a.source_hash
    r["command"] = a.cmd
    d = json.load(open(a.json)) if os.path.exists(a.json) else {}
    d[a.key] = r
    with open(a.json, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    print(f"| {a.key} | `{r['kernel'][:60]}` | FETCH {r['fetch_kib']:.0f} KiB x {r['fetch_scale']:.4f} | "
          f"WRITE {r['write_kib']:.0f} KiB x {r['write_scale']:.4f} | {r['bytes_per_launch'] / 1e9:.3f} GB |")


if __name__ == "__main__":
    main()
