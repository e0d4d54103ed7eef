"""Short text summaries of rocprofv3 output for the tdsolve kernels.

    stats    per-kernel calls and average duration from a
             `rocprofv3 --kernel-trace --stats --output-format csv` run;
    traffic  HBM bytes per dispatch of one kernel from two
             `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs, each
             scaled by what the same counter reads for a plain streaming
             kernel of known size (a torch elementwise negation that reads and
             writes the same number of bytes) in the same run;
    path     the same for every kernel of one step of the path, and the sum.

The traffic summary records a SHA-256 of the kernel sources and build flags;
bench.py reports the figure only while that hash still matches the tree.

    python -m paper_0901_2859_amd.profdigest stats DIR --cmd "..." --out FILE
    python -m paper_0901_2859_amd.profdigest traffic --fetch DIR --write DIR \\
        --kernel SUBSTR --copy-kernel SUBSTR --copy-bytes B --cmd "..." --out FILE
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/tds_kernels.hip", "csrc/tds_internal.h", "build.py"]


def source_hash() -> str:
    """SHA-256 over the files that define the device code of the solve."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(rel.encode() + b"\0" + f.read() + b"\0")
    return h.hexdigest()


def _find(d: str, suffix: str) -> str:
    hits = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not hits:
        raise FileNotFoundError(f"no *{suffix} under {d}")
    return hits[-1]


def short_name(name: str) -> str:
    """`void tds::k_sweep_reg<64, float, double, 1>(...)` -> `k_sweep_reg<64, float, double, 1>`."""
    n = name.split("(")[0]
    if n.startswith("void "):
        n = n[5:]
    return n.replace("tds::", "")


def kernel_stats(d: str):
    rows = []
    with open(_find(d, "kernel_stats.csv"), newline="") as f:
        for r in csv.DictReader(f):
            rows.append((short_name(r["Name"]), int(r["Calls"]), float(r["AverageNs"]),
                         float(r["MinNs"]), float(r["MaxNs"]), float(r["Percentage"])))
    return rows


def counter_values(d: str, counter: str):
    """{kernel short name: [value per dispatch]} for one counter."""
    out: dict[str, list[float]] = {}
    with open(_find(d, "counter_collection.csv"), newline="") as f:
        for r in csv.DictReader(f):
            if r.get("Counter_Name") != counter:
                continue
            out.setdefault(short_name(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
    return out


def _pick(table, sub: str):
    keys = [k for k in table if sub in k]
    if not keys:
        raise KeyError(f"no kernel matching {sub!r} in {sorted(table)}")
    # the most frequent match is the timed kernel
    return max(keys, key=lambda k: len(table[k]))


def cmd_stats(a):
    rows = kernel_stats(a.dir)
    lines = [f"# rocprofv3 kernel statistics", f"# command: {a.cmd}", "",
             f"{'kernel':<58} {'calls':>6} {'avg_us':>9} {'min_us':>9} {'max_us':>9} {'pct':>6}"]
    for name, calls, avg, mn, mx, pct in rows:
        lines.append(f"{name[:58]:<58} {calls:>6} {avg / 1e3:>9.2f} {mn / 1e3:>9.2f} "
                     f"{mx / 1e3:>9.2f} {pct:>6.2f}")
    text = "\n".join(lines) + "\n"
    _emit(text, a.out)


def cmd_traffic(a):
    fetch = counter_values(a.fetch, "FETCH_SIZE")
    write = counter_values(a.write, "WRITE_SIZE")
    kf, kw = _pick(fetch, a.kernel), _pick(write, a.kernel)
    cf, cw = _pick(fetch, a.copy_kernel), _pick(write, a.copy_kernel)
    f_k, w_k = statistics.median(fetch[kf]), statistics.median(write[kw])
    f_c, w_c = statistics.median(fetch[cf]), statistics.median(write[cw])
    # the copy reads and writes copy_bytes: counter KiB -> bytes factors
    sf = a.copy_bytes / (f_c * 1024.0)
    sw = a.copy_bytes / (w_c * 1024.0)
    traffic = f_k * 1024.0 * sf + w_k * 1024.0 * sw
    lines = [
        "# HBM traffic per dispatch from rocprofv3 --pmc (FETCH_SIZE, WRITE_SIZE; KiB)",
        f"# fetch command: {a.cmd_fetch}",
        f"# write command: {a.cmd_write}",
        f"kernel={kf}",
        f"source_sha256={source_hash()}",
        f"dispatches_fetch={len(fetch[kf])}",
        f"dispatches_write={len(write[kw])}",
        f"fetch_kib_per_dispatch={f_k:.1f}",
        f"write_kib_per_dispatch={w_k:.1f}",
        f"copy_kernel={cf}",
        f"copy_bytes={a.copy_bytes}",
        f"copy_fetch_kib={f_c:.1f}",
        f"copy_write_kib={w_c:.1f}",
        f"fetch_scale={sf:.4f}",
        f"write_scale={sw:.4f}",
        f"traffic_bytes_per_launch={traffic:.0f}",
    ]
    if a.alg_bytes:
        lines.append(f"algorithmic_bytes_per_launch={a.alg_bytes}")
        lines.append(f"traffic_over_algorithmic={traffic / a.alg_bytes:.4f}")
    _emit("\n".join(lines) + "\n", a.out)


def cmd_path(a):
    """HBM traffic of one step of the path: the per-dispatch traffic of each
    kernel of the step (substrings in --kernels, each launched once per
    step), scaled as in cmd_traffic, and their sum."""
    fetch = counter_values(a.fetch, "FETCH_SIZE")
    write = counter_values(a.write, "WRITE_SIZE")
    cf, cw = _pick(fetch, a.copy_kernel), _pick(write, a.copy_kernel)
    sf = a.copy_bytes / (statistics.median(fetch[cf]) * 1024.0)
    sw = a.copy_bytes / (statistics.median(write[cw]) * 1024.0)
    lines = [
        "# HBM traffic of one step of the path from rocprofv3 --pmc (FETCH_SIZE, WRITE_SIZE),",
        "# each kernel's median per dispatch scaled by the plain copy's counters",
        f"# fetch command: {a.cmd_fetch}",
        f"# write command: {a.cmd_write}",
        f"source_sha256={source_hash()}",
        f"fetch_scale={sf:.4f}",
        f"write_scale={sw:.4f}",
    ]
    total_f = total_w = 0.0
    for sub in a.kernels.split(";"):
        kf, kw = _pick(fetch, sub), _pick(write, sub)
        fb = statistics.median(fetch[kf]) * 1024.0 * sf
        wb = statistics.median(write[kw]) * 1024.0 * sw
        total_f += fb
        total_w += wb
        lines.append(f"kernel={kf} fetch_bytes={fb:.0f} write_bytes={wb:.0f}")
    lines.append(f"path_fetch_bytes_per_step={total_f:.0f}")
    lines.append(f"path_write_bytes_per_step={total_w:.0f}")
    lines.append(f"path_traffic_bytes_per_step={total_f + total_w:.0f}")
    if a.alg_bytes:
        lines.append(f"algorithmic_bytes_per_step={a.alg_bytes}")
        lines.append(f"traffic_over_algorithmic={(total_f + total_w) / a.alg_bytes:.4f}")
    _emit("\n".join(lines) + "\n", a.out)


def read_traffic(path: str):
    """(traffic bytes per launch, kernel) from a traffic summary, or None when
    the file is absent or was taken from other kernel sources."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.startswith("#"):
                k, v = line.strip().split("=", 1)
                kv[k] = v
    if kv.get("source_sha256") != source_hash():
        return None
    return float(kv["traffic_bytes_per_launch"]), kv.get("kernel", "")


def _emit(text: str, out: str | None):
    if out:
        with open(out, "w") as f:
            f.write(text)
    print(text, end="")


def main(argv=None):
    p = argparse.ArgumentParser(prog="profdigest")
    sub = p.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("dir")
    s.add_argument("--cmd", default="")
    s.add_argument("--out")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--kernel", required=True)
    t.add_argument("--copy-kernel", required=True)
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--alg-bytes", type=int, default=0)
    t.add_argument("--cmd-fetch", default="")
    t.add_argument("--cmd-write", default="")
    t.add_argument("--out")
    q = sub.add_parser("path")
    q.add_argument("--fetch", required=True)
    q.add_argument("--write", required=True)
    q.add_argument("--kernels", required=True, help="kernel name substrings separated by semicolons")
    q.add_argument("--copy-kernel", required=True)
    q.add_argument("--copy-bytes", type=int, required=True)
    q.add_argument("--alg-bytes", type=int, default=0)
    q.add_argument("--cmd-fetch", default="")
    q.add_argument("--cmd-write", default="")
    q.add_argument("--out")
    a = p.parse_args(argv)
    if a.what == "stats":
        cmd_stats(a)
    elif a.what == "path":
        cmd_path(a)
    else:
        cmd_traffic(a)


if __name__ == "__main__":
    main()
