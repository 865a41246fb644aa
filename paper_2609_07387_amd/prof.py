"""rocprofv3 result helpers: kernel-time summaries and measured HBM traffic.

Measured traffic of a kernel comes from two counter runs of the same command
(FETCH_SIZE, then WRITE_SIZE; KiB per dispatch).  Each counter is scaled by
what it reads for a plain device copy of known size in the same run (the
benchmark issues one 256 MiB copy outside its timed region): the counters
count fixed-size requests, and the copy tells how many bytes one counted
unit is.  The stored record (a short markdown file with the figures and a
JSON block) carries a digest of the kernel sources; once the sources change
the record no longer applies and the benchmark reports no traffic.

  python -m paper_2609_07387_amd.prof stats KERNEL_STATS_CSV TITLE COMMAND [TRACE_CSV LABEL=K1|K2=N ...] > profiles/NAME.md
  python -m paper_2609_07387_amd.prof traffic FETCH_CSV WRITE_CSV K1[|K2...] COPY_BYTES COMMAND OUT_MD [N_LAST]
      [--sizes READREQ_CSV,WRITEREQ_CSV] [--exclude FILE[,FILE...]]
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_KERNEL = "copyBuffer"


def _code_only(text: str) -> str:
    """C++ source without comments and blank space, so that a record stays
    valid across edits that change no code.  String and character literals
    are kept whole."""
    out, i, n = [], 0, len(text)
    while i < n:
        ch = text[i]
        if text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        elif ch in "\"'":
            j = i + 1
            while j < n and text[j] != ch:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            out.append(ch)
            i += 1
    return " ".join("".join(out).split())


def source_digest(exclude=()) -> str:
    """sha256 over the code (comments and spacing removed) of the device and
    host sources of libucns.  exclude: file names left out, for a record whose
    kernels take no code from them (a header that only defines other
    kernels)."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(HERE, "csrc", "*"))):
        if os.path.basename(p) in exclude:
            continue
        if p.endswith((".hip", ".hpp", ".cpp", ".h")):
            with open(p, encoding="utf-8") as f:
                h.update(os.path.basename(p).encode())
                h.update(_code_only(f.read()).encode())
    return h.hexdigest()


def _by_kernel(path, counter):
    """Counter values per kernel name, in dispatch order."""
    vals = {}
    with open(path) as f:
        rows = [r for r in csv.DictReader(f) if r["Counter_Name"] == counter]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    for r in rows:
        vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return vals


def _mean_by_kernel(path, counter, n_last=0):
    """Mean per kernel over all dispatches, or over the last n_last."""
    out = {}
    for k, v in _by_kernel(path, counter).items():
        w = v[-n_last:] if n_last else v
        out[k] = (sum(w) / len(w), len(w))
    return out


def _copy_reading(path, counter):
    """The calibration copy is the largest copy dispatch of the run (others
    are small host uploads)."""
    hits = [v for k, v in _by_kernel(path, counter).items() if COPY_KERNEL in k]
    if not hits:
        raise SystemExit(f"no {COPY_KERNEL} dispatch in {path}")
    return max(max(v) for v in hits)


def _pick(d, sub):
    hits = [k for k in d if sub in k]
    if len(hits) != 1:
        raise SystemExit(f"kernel '{sub}': {len(hits)} matches in {sorted(d)}")
    return hits[0], d[hits[0]]


# Request counters of the memory side of L2 (one run for reads, one for
# writes; each within the four-counter limit of that block).
READ_REQ = ("TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_BUBBLE_sum", "TCC_EA0_RDREQ_DRAM_sum")
WRITE_REQ = ("TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum", "TCC_EA0_WRREQ_DRAM_sum")


def _sum_means(path, counter, kernel, n_last):
    d = _mean_by_kernel(path, counter, n_last)
    return sum(_pick(d, sub)[1][0] for sub in kernel.split("|"))


def request_sizes(read_csv, write_csv, kernel, copy_bytes, n_last=0):
    """Read and write bytes from request counts by size: 32-byte reads
    (RDREQ_32B) count 32 B; every other read request counts the bytes one
    request moved in the calibration copy (copy bytes / its read requests);
    64-byte writes (WRREQ_64B) count 64 B and the other writes 32 B, checked
    against the copy's known write size.  Also the share of read requests that
    went to DRAM."""
    r = {c: _sum_means(read_csv, c, kernel, n_last) for c in READ_REQ}
    w = {c: _sum_means(write_csv, c, kernel, n_last) for c in WRITE_REQ}
    cr = {c: _copy_reading(read_csv, c) for c in READ_REQ}
    cw = {c: _copy_reading(write_csv, c) for c in WRITE_REQ}
    big = cr["TCC_EA0_RDREQ_sum"] - cr["TCC_EA0_RDREQ_32B_sum"]
    per_req = (copy_bytes - 32.0 * cr["TCC_EA0_RDREQ_32B_sum"]) / big
    read_b = 32.0 * r["TCC_EA0_RDREQ_32B_sum"] + per_req * (r["TCC_EA0_RDREQ_sum"] - r["TCC_EA0_RDREQ_32B_sum"])

    def wbytes(d):
        return 64.0 * d["TCC_EA0_WRREQ_64B_sum"] + 32.0 * (d["TCC_EA0_WRREQ_sum"] - d["TCC_EA0_WRREQ_64B_sum"])

    return {"read_requests": r, "write_requests": w, "copy_read_requests": cr, "copy_write_requests": cw,
            "copy_bytes_per_read_request": per_req, "copy_write_bytes_from_sizes": wbytes(cw),
            "read_bytes": read_b, "write_bytes": wbytes(w), "bytes_per_launch": read_b + wbytes(w),
            "dram_read_share": r["TCC_EA0_RDREQ_DRAM_sum"] / max(r["TCC_EA0_RDREQ_sum"], 1.0)}


def traffic(fetch_csv, write_csv, kernel, copy_bytes, command, n_last=0, exclude=(), sizes=None):
    """kernel: one name substring, or several joined by '|' (the kernels of
    one library call; their per-dispatch means are summed).  n_last: average
    the last n dispatches only (the window a benchmark times).  sizes: the
    (read, write) request-counter CSVs of the same command, for a second
    estimate from request sizes."""
    fe = _mean_by_kernel(fetch_csv, "FETCH_SIZE", n_last)
    wr = _mean_by_kernel(write_csv, "WRITE_SIZE", n_last)
    names, f_kib, w_kib, nf, nw = [], 0.0, 0.0, [], []
    for sub in kernel.split("|"):
        name, (fk, n1) = _pick(fe, sub)
        _, (wk, n2) = _pick(wr, sub)
        names.append(name)
        f_kib += fk
        w_kib += wk
        nf.append(n1)
        nw.append(n2)
    name = " + ".join(names)
    cf_kib = _copy_reading(fetch_csv, "FETCH_SIZE")
    cw_kib = _copy_reading(write_csv, "WRITE_SIZE")
    f_scale = copy_bytes / (cf_kib * 1024.0)
    w_scale = copy_bytes / (cw_kib * 1024.0)
    fetch_b = f_kib * 1024.0 * f_scale
    write_b = w_kib * 1024.0 * w_scale
    return {"kernel": name, "dispatches": [nf, nw], "fetch_kib": f_kib, "write_kib": w_kib,
            "copy_bytes": copy_bytes, "copy_fetch_kib": cf_kib, "copy_write_kib": cw_kib,
            "fetch_scale": f_scale, "write_scale": w_scale, "fetch_bytes": fetch_b, "write_bytes": write_b,
            "bytes_per_launch": fetch_b + write_b, "window_last_dispatches": n_last,
            "by_request_size": request_sizes(sizes[0], sizes[1], kernel, copy_bytes, n_last) if sizes else None,
            "digest_exclude": list(exclude), "source_digest": source_digest(exclude), "command": command}


def traffic_md(rec):
    return "\n".join([
        f"# Measured HBM traffic: `{rec['kernel'][:100]}`", "",
        "Command (two runs, one counter each):", "", "```", rec["command"], "```", "",
        "| counter | KiB / dispatch | copy kernel KiB ({:.0f} MiB copied) | scale | bytes / launch |".format(
            rec["copy_bytes"] / 2**20),
        "|---|---|---|---|---|",
        f"| FETCH_SIZE | {rec['fetch_kib']:.1f} | {rec['copy_fetch_kib']:.1f} | {rec['fetch_scale']:.3f} | "
        f"{rec['fetch_bytes']:.4g} |",
        f"| WRITE_SIZE | {rec['write_kib']:.1f} | {rec['copy_write_kib']:.1f} | {rec['write_scale']:.3f} | "
        f"{rec['write_bytes']:.4g} |", "",
        f"Total per launch: {rec['bytes_per_launch']:.4g} bytes"
        + (f" (mean of the last {rec['window_last_dispatches']} dispatches of each kernel)."
           if rec.get("window_last_dispatches") else " (mean over all dispatches)."), ""]
        + (_sizes_md(rec["by_request_size"]) if rec.get("by_request_size") else [])
        + ["```json", json.dumps(rec, indent=1), "```", ""])


def _sizes_md(z):
    r, w = z["read_requests"], z["write_requests"]
    return [
        "By request size (separate runs: " + ", ".join(READ_REQ) + "; then " + ", ".join(WRITE_REQ) + "):", "",
        "| | requests / launch | of which 32 B (reads) or 64 B (writes) | to DRAM | bytes / launch |",
        "|---|---|---|---|---|",
        f"| reads | {r['TCC_EA0_RDREQ_sum']:.4g} | {r['TCC_EA0_RDREQ_32B_sum']:.4g} | "
        f"{r['TCC_EA0_RDREQ_DRAM_sum']:.4g} | {z['read_bytes']:.4g} |",
        f"| writes | {w['TCC_EA0_WRREQ_sum']:.4g} | {w['TCC_EA0_WRREQ_64B_sum']:.4g} | "
        f"{w['TCC_EA0_WRREQ_DRAM_sum']:.4g} | {z['write_bytes']:.4g} |", "",
        f"Other read requests are counted at the calibration copy's {z['copy_bytes_per_read_request']:.1f} B per "
        f"request; the copy's writes by size come to {z['copy_write_bytes_from_sizes']:.4g} B. "
        f"Total by request size: {z['bytes_per_launch']:.4g} bytes per launch "
        f"(TCC_BUBBLE {r['TCC_BUBBLE_sum']:.4g} per launch).", ""]


def load_traffic(path):
    """The stored record if it was taken on the current kernel sources, else None."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        text = f.read()
    i = text.find("```json")
    if i < 0:
        return None
    rec = json.loads(text[i + 7:text.index("```", i + 7)])
    return rec if rec.get("source_digest") == source_digest(tuple(rec.get("digest_exclude", ()))) else None


def last_calls_us(trace_csv, kernel, n):
    """Mean duration (us) of the last n dispatches of each kernel in `kernel`
    ('|'-joined substrings), and their sum: the window a benchmark times."""
    rows = list(csv.DictReader(open(trace_csv)))
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    parts = []
    for sub in kernel.split("|"):
        d = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows if sub in r["Kernel_Name"]]
        if len(d) < n:
            raise SystemExit(f"kernel '{sub}': {len(d)} dispatches, fewer than {n}")
        parts.append((sub, sum(d[-n:]) / n))
    return parts, sum(p[1] for p in parts)


def stats_md(stats_csv, title, command, top=14, trace_csv=None, windows=()):
    rows = list(csv.DictReader(open(stats_csv)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out = [f"# {title}", "", "Command:", "", "```", command, "```", "",
           "| kernel | calls | avg us | min us | max us | % time |", "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        out.append(f"| `{r['Name'][:110]}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                   f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    for label, kernel, n in windows:
        parts, total = last_calls_us(trace_csv, kernel, n)
        out += ["", f"**{label}** (mean of the last {n} dispatches of each kernel): "
                + " + ".join(f"`{k}` {t:.1f} us" for k, t in parts) + f" = **{total:.1f} us** per call."]
    return "\n".join(out) + "\n"


def main(argv):
    if len(argv) >= 4 and argv[0] == "stats":
        # optional trailing args: TRACE_CSV then LABEL=KERNELS=N ...
        trace = argv[4] if len(argv) > 4 else None
        wins = [tuple(w.split("=")) for w in argv[5:]]
        wins = [(lab, ker, int(n)) for lab, ker, n in wins]
        sys.stdout.write(stats_md(argv[1], argv[2], argv[3], trace_csv=trace, windows=wins))
    elif len(argv) >= 7 and argv[0] == "traffic":
        opts, pos = {}, []
        it = iter(argv[1:])
        for a in it:
            if a in ("--exclude", "--sizes"):
                opts[a] = next(it)
            else:
                pos.append(a)
        excl = tuple(x for x in opts.get("--exclude", "").split(",") if x)
        sizes = tuple(opts["--sizes"].split(",")) if "--sizes" in opts else None
        rec = traffic(pos[0], pos[1], pos[2], float(pos[3]), pos[4], int(pos[6]) if len(pos) > 6 else 0,
                      exclude=excl, sizes=sizes)
        with open(pos[5], "w") as f:
            f.write(traffic_md(rec))
        print(json.dumps(rec))
    else:
        sys.stderr.write(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
