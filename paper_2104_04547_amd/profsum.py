"""Condense rocprofv3 results (its SQLite `*_results.db` output) into short text.

  stats    per-kernel dispatch statistics of a --kernel-trace run (calls, total
           and average duration, share), kernels named as the library's timing
           keys (conv kernels by variant).
  traffic  HBM bytes per dispatch of one kernel from two --pmc runs (FETCH_SIZE,
           WRITE_SIZE), each scaled by what the same counter reads for a plain
           elementwise copy of known size (two more --pmc runs of
           `bench.py --copy-probe MIB`); optionally merges an entry into the JSON
           the benchmark reads to fill its roofline `traffic` field, keyed by the
           benchmark's kernel name and tied to the SHA-256 of the kernel's source.

  python -m paper_2104_04547_amd.profsum stats RESULTS.db --command "CMD" [--top N]
  python -m paper_2104_04547_amd.profsum traffic --kernel NAME --key BENCH_NAME --source FILE.hip \\
      --fetch F.db --write W.db --copy-fetch CF.db --copy-write CW.db --copy-mib MIB [--json OUT] \\
      --command "CMD" ...
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sqlite3
import subprocess
import sys
from collections import defaultdict
from typing import Dict, List

HERE = os.path.dirname(os.path.abspath(__file__))


def demangle(names: List[str]) -> Dict[str, str]:
    mangled = [n for n in names if n.startswith("_Z")]
    out = {n: n for n in names}
    if mangled:
        try:
            r = subprocess.run(["c++filt"], input="\n".join(mangled), capture_output=True, text=True, check=True)
            for m, d in zip(mangled, r.stdout.splitlines()):
                out[m] = d
        except (OSError, subprocess.CalledProcessError):
            pass
    return out


_CONV8 = re.compile(r"k_conv8<(\d+), (\d+), (\d+), (\d+), (\d+), (\d+), (\d+)(?:, (\d+))?(?:, (\d+))?>")
_CONV = re.compile(r"k_conv<([^,]+), (\d+), (\d+), (\d+), (\d+), (\d+), (\d+), (\d+)>")
_PLAIN = re.compile(r"(?:cf::\(anonymous namespace\)::)?(k_\w+)")


_MANGLED_CONV = re.compile(r"k_conv([48]?)I(DF16b|f)?((?:Li\d+E)+)E")
_CONV4 = re.compile(r"k_conv4<(\d+), (\d+), (\d+), (\d+), (\d+), (\d+), (\d+)>")


def _split(wn: int) -> str:
    """Column split of the tap-pair conv as in the library's variant names."""
    return f"c{wn}" if wn > 1 else ""


def _poses(pp: int) -> str:
    """Poses per workgroup of the tap-pair conv as in the library's variant names."""
    return f"_p{pp}" if pp > 1 else ""


def short_name(name: str) -> str:
    """Conv kernels as 'conv.<variant>' (the library's timing keys; 'conv.f32.' for
    the float32 instances), other library kernels by function name."""
    m = _MANGLED_CONV.search(name)
    if m:   # names c++filt leaves mangled (bfloat16 template arguments)
        p8, t, ints = m.groups()
        v = [int(x) for x in re.findall(r"Li(\d+)E", ints)]
        if len(v) in (7, 8, 9):
            ks, s, tz, ty, tx, nw, nt = v[:7]
            wn = v[7] if len(v) >= 8 else 1
            pp = v[8] if len(v) == 9 else 1
            pre = {"8": "conv.p8", "4": "conv.q4"}.get(p8) or ("conv.f32." if t == "f" else "conv.")
            return f"{pre}k{ks}s{s}_t{tz}x{ty}x{tx}_w{nw}{_split(wn)}_n{nt}{_poses(pp)}"
    m = _CONV4.search(name)
    if m:
        ks, s, tz, ty, tx, nw, nt = m.groups()
        return f"conv.q4k{ks}s{s}_t{tz}x{ty}x{tx}_w{nw}_n{nt}"
    m = _CONV8.search(name)
    if m:
        ks, s, tz, ty, tx, nw, nt, wn, pp = m.groups()
        return f"conv.p8k{ks}s{s}_t{tz}x{ty}x{tx}_w{nw}{_split(int(wn or 1))}_n{nt}{_poses(int(pp or 1))}"
    m = _CONV.search(name)
    if m:
        t, ks, s, tz, ty, tx, nw, nt = m.groups()
        pre = "conv.f32." if t.strip() == "float" else "conv."
        return f"{pre}k{ks}s{s}_t{tz}x{ty}x{tx}_w{nw}_n{nt}"
    if "cf::" in name:
        m = _PLAIN.search(name.split("cf::", 1)[1])
        if m:
            return m.group(1)
    m = re.search(r"\d(k_[A-Za-z0-9_]+?)I", name) if name.startswith("_Z") else None
    return m.group(1) if m else name[:80]


def kernel_rows(db: str):
    con = sqlite3.connect(db)
    rows = con.execute("SELECT name, start, end, grid_x * grid_y * grid_z FROM kernels").fetchall()
    con.close()
    names = demangle(sorted({r[0] for r in rows}))
    return [(short_name(names[n]), int(e) - int(s), int(g)) for n, s, e, g in rows]


def stats(db: str, top: int) -> List[dict]:
    """Per kernel: all dispatches, and the full-size ones alone (largest grid of
    that kernel -- the launches of whole chunks, without tuning probes or small
    checks)."""
    per = defaultdict(list)
    for name, dur, grid in kernel_rows(db):
        per[name].append((dur, grid))
    total = sum(d for v in per.values() for d, _ in v) or 1
    out = []
    for k, v in per.items():
        ns = sum(d for d, _ in v)
        gmax = max(g for _, g in v)
        full = [d for d, g in v if g == gmax]
        out.append(dict(kernel=k, calls=len(v), total_ms=ns / 1e6, avg_ms=ns / len(v) / 1e6, share=ns / total,
                        calls_full=len(full), avg_full_ms=sum(full) / len(full) / 1e6))
    out.sort(key=lambda r: -r["total_ms"])
    return out[:top]


def counter_per_dispatch(db: str, counter: str, full_only: bool = True) -> Dict[str, List[float]]:
    """Counter value per dispatch, per kernel (full-size dispatches only: the
    largest grid of each kernel)."""
    con = sqlite3.connect(db)
    rows = con.execute("SELECT kernel_name, dispatch_id, grid_size, value FROM counters_collection "
                       "WHERE counter_name = ?", (counter,)).fetchall()
    con.close()
    names = demangle(sorted({r[0] for r in rows}))
    per = defaultdict(dict)
    for n, d, g, v in rows:
        k = short_name(names[n])
        val, _ = per[k].get(d, (0.0, g))
        per[k][d] = (val + float(v), int(g))
    out = {}
    for k, v in per.items():
        gmax = max(g for _, g in v.values())
        out[k] = [val for val, g in v.values() if g == gmax or not full_only]
    return out


def copy_factor(db: str, counter: str, nbytes: int) -> float:
    """Counter reading (KiB) of the largest elementwise dispatch / the bytes it must move."""
    per = counter_per_dispatch(db, counter)
    vals = [max(v) for k, v in per.items() if "elementwise" in k or "copy" in k.lower()]
    if not vals:
        raise SystemExit(f"no copy kernel found in {db}")
    return max(vals) * 1024.0 / nbytes


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="mode", required=True)
    s = sub.add_parser("stats")
    s.add_argument("db")
    s.add_argument("--top", type=int, default=25)
    s.add_argument("--command", required=True)
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True)
    t.add_argument("--key", default="", help="the benchmark's name of the kernel (default: --kernel)")
    t.add_argument("--source", default="cf_conv.hip", help="source file of the kernel under csrc/")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-mib", type=int, required=True)
    t.add_argument("--algorithmic-bytes", type=float, default=0.0)
    t.add_argument("--json", default="")
    t.add_argument("--command", action="append", required=True)
    a = ap.parse_args(argv)

    if a.mode == "stats":
        rows = stats(a.db, a.top)
        print(f"# rocprofv3 kernel-trace summary\n# command: {a.command}\n#")
        print("# full = dispatches with the kernel's largest grid (whole chunks)")
        print(f"{'kernel':<36} {'calls':>6} {'total_ms':>10} {'avg_ms':>9} {'share':>7} {'full':>5} {'avg_full_ms':>11}")
        for r in rows:
            print(f"{r['kernel']:<36} {r['calls']:>6} {r['total_ms']:>10.3f} {r['avg_ms']:>9.4f} {r['share']:>7.2%} "
                  f"{r['calls_full']:>5} {r['avg_full_ms']:>11.4f}")
        return

    nbytes = a.copy_mib << 20
    # the copy reads and writes nbytes each
    f_fac = copy_factor(a.copy_fetch, "FETCH_SIZE", nbytes)
    w_fac = copy_factor(a.copy_write, "WRITE_SIZE", nbytes)
    fetch = counter_per_dispatch(a.fetch, "FETCH_SIZE").get(a.kernel)
    write = counter_per_dispatch(a.write, "WRITE_SIZE").get(a.kernel)
    if not fetch or not write:
        raise SystemExit(f"kernel {a.kernel} not found in the counter runs")
    fb = sum(fetch) / len(fetch) * 1024.0 / f_fac
    wb = sum(write) / len(write) * 1024.0 / w_fac
    src = os.path.join(HERE, "csrc", a.source)
    res = dict(kernel=a.kernel, dispatches=[len(fetch), len(write)], fetch_bytes_per_launch=fb,
               write_bytes_per_launch=wb, copy_factor_fetch=f_fac, copy_factor_write=w_fac,
               copy_bytes=nbytes, commands=a.command, source=a.source,
               source_sha256=hashlib.sha256(open(src, "rb").read()).hexdigest())
    if a.algorithmic_bytes:
        res["algorithmic_bytes_per_launch"] = a.algorithmic_bytes
    print(f"# HBM traffic per dispatch of {a.kernel} (rocprofv3 --pmc, scaled by a plain copy)")
    for c in a.command:
        print(f"# command: {c}")
    print(f"copy probe: {nbytes} B read + written; FETCH_SIZE reads {f_fac:.4f} x, WRITE_SIZE {w_fac:.4f} x")
    print(f"{a.kernel}: {len(fetch)} dispatches; fetched {fb / 1e6:.2f} MB, written {wb / 1e6:.2f} MB per launch "
          f"(raw {sum(fetch) / len(fetch) / 1024:.1f} / {sum(write) / len(write) / 1024:.1f} MiB)")
    if a.json:
        allt = json.load(open(a.json)) if os.path.exists(a.json) else {}
        allt[a.key or a.kernel] = res
        json.dump(allt, open(a.json, "w"), indent=1)


if __name__ == "__main__":
    sys.exit(main())
