"""Summaries of rocprofv3 result databases for the profiles/ folder.

    python -m paper_2304_09180_amd.profsum trace  RUN_DIR  "COMMAND"            > profiles/<name>.md
    python -m paper_2304_09180_amd.profsum traffic FETCH_DIR WRITE_DIR CFETCH_DIR CWRITE_DIR KERNEL BYTES "CMDS"

The traffic summary scales each kernel counter by what the same counter reads for
a plain device copy of known size, and records a hash of the kernel sources so a
reader (bench.py) can tell whether the counters still describe the current code.
"""
from __future__ import annotations

import glob
import hashlib
import os
import re
import sqlite3
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def source_hash() -> str:
    h = hashlib.sha256()
    # the kernel sources and the build script (its compiler flags shape the code too)
    for p in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))) + [os.path.join(HERE, "build.py")]:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _db(d):
    return sqlite3.connect(glob.glob(os.path.join(d, "*.db"))[0])


def _short(n):
    n = re.sub(r"^void ", "", n)
    n = n.replace("clot::", "").replace("(anonymous namespace)::", "")
    return re.sub(r"\(.*$", "", n)[:70]


def trace(run_dir, cmd, top=25):
    cur = _db(run_dir).cursor()
    rows = cur.execute("select name, count(*), sum(duration), avg(duration) from kernels group by name "
                       "order by sum(duration) desc").fetchall()
    tot = sum(r[2] for r in rows)
    out = [f"command: `{cmd}`", f"kernel source hash: {source_hash()}", "",
           "| kernel | calls | total ms | avg us | share |", "|---|---:|---:|---:|---:|"]
    for r in rows[:top]:
        out.append(f"| `{_short(r[0])}` | {r[1]} | {r[2] / 1e6:.3f} | {r[3] / 1e3:.2f} | {100 * r[2] / tot:.1f}% |")
    out.append(f"| all kernels | {sum(r[1] for r in rows)} | {tot / 1e6:.3f} | | 100% |")
    return "\n".join(out)


def _avg(d, pat):
    cur = _db(d).cursor()
    vals = [r[0] for r in cur.execute("select value from counters_collection where kernel_name like ?",
                                      (f"%{pat}%",)).fetchall()]
    return sum(vals) / len(vals), len(vals)


def traffic(fetch, write, cfetch, cwrite, kernel, algo_bytes, cmds):
    copy_kib = 256 * 1024.0
    cf, _ = _avg(cfetch, "copyBuffer")
    cw, _ = _avg(cwrite, "copyBuffer")
    kf, nf = _avg(fetch, kernel)
    kw, nw = _avg(write, kernel)
    ffac, wfac = copy_kib / cf, copy_kib / cw
    tb = (kf * ffac + kw * wfac) * 1024.0
    lines = [f"commands: {cmds}", f"kernel source hash: {source_hash()}", f"kernel: `{kernel}`", "",
             f"copy calibration (256 MiB device copy): FETCH_SIZE {cf:.1f} KiB -> factor {ffac:.4f}; "
             f"WRITE_SIZE {cw:.1f} KiB -> factor {wfac:.4f}",
             f"kernel FETCH_SIZE {kf:.1f} KiB/dispatch over {nf} dispatches; WRITE_SIZE {kw:.1f} KiB/dispatch over {nw}",
             f"algorithmic bytes per launch: {int(algo_bytes)}",
             f"traffic_bytes_per_launch: {int(tb)}",
             f"traffic / algorithmic: {tb / algo_bytes:.3f}"]
    return "\n".join(lines)


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        print(trace(sys.argv[2], sys.argv[3]))
    elif sys.argv[1] == "traffic":
        print(traffic(*sys.argv[2:7], float(sys.argv[7]), sys.argv[8]))
    elif sys.argv[1] == "hash":
        print(source_hash())
