"""HBM traffic of the Ozaki-II kernels from rocprofv3 counter runs.

Two runs of the same command, one with ``--pmc FETCH_SIZE`` and one with
``--pmc WRITE_SIZE`` (the counters read KiB per dispatch), each also timing a
plain device copy of known size (``bench.py --copy-calibration-mib N``).
Per kernel family the mean counter value per dispatch is scaled by
(known copy bytes) / (counter value of the copy) -- one factor for reads,
one for writes -- and reported as bytes per launch, next to the sha256 of
the kernel sources it was measured on.  bench.py uses the figures only while
that source is unchanged.

    python -m paper_2609_29554_amd.pmc FETCH.csv WRITE.csv COPY_MIB OUT.md "command"

It also writes the kernel-time summaries of ``rocprofv3 --kernel-trace
--stats`` runs (``python -m paper_2609_29554_amd.pmc trace ...``) and the
VALU activity of a ``rocprofv3 --pmc VALUBusy SQ_INSTS_VALU SQ_WAVES`` run
(``python -m paper_2609_29554_amd.pmc valu ...``).
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sqlite3
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
# the device code of the Ozaki-II kernels (a change to the host-side plane
# padding in ozii.cpp also calls for new counter runs)
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in
                  ("k_ozaki.hip", "k_limbs.hip", "ozii_elem.hpp", "ozii_bytes.hpp",
                   "ozii_stage.hpp", "expansion.hpp")]
_KNAME = re.compile(r"(?:^|::|\s)(k_[A-Za-z0-9_]+)\s*(<[^()]*>)?\s*\(")


def source_sha() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _family(name: str):
    """Base name of one of this library's kernels (k_...), else None."""
    m = _KNAME.search(name)
    return m.group(1) if m else None


def short_name(name: str) -> str:
    """Kernel name without namespace and argument list, template arguments kept."""
    m = _KNAME.search(name)
    if m:
        return m.group(1) + (m.group(2) or "")
    return name.split("(")[0].strip()


def _read(path: str, counter: str):
    per = defaultdict(list)
    copies = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        v = float(r["Counter_Value"])
        fam = _family(r["Kernel_Name"])
        if fam:
            per[fam].append(v)
        elif "copy" in r["Kernel_Name"].lower() or "elementwise" in r["Kernel_Name"]:
            copies.append(v)
    return per, copies


def summarize(fetch_csv: str, write_csv: str, copy_mib: float):
    f_per, f_copy = _read(fetch_csv, "FETCH_SIZE")
    w_per, w_copy = _read(write_csv, "WRITE_SIZE")
    want_kib = copy_mib * 1024.0
    # the calibration copy is the largest copy-like dispatch of each run
    ff = want_kib / max(f_copy) if f_copy else None
    fw = want_kib / max(w_copy) if w_copy else None
    out = {}
    for fam in sorted(set(f_per) | set(w_per)):
        fk = sum(f_per[fam]) / len(f_per[fam]) if f_per.get(fam) else None
        wk = sum(w_per[fam]) / len(w_per[fam]) if w_per.get(fam) else None
        rec = {"dispatches": max(len(f_per.get(fam, [])), len(w_per.get(fam, []))),
               "fetch_kib_per_launch": fk, "write_kib_per_launch": wk}
        if fk is not None and wk is not None and ff and fw:
            rec["hbm_bytes_per_launch"] = (fk * ff + wk * fw) * 1024.0
        out[fam] = rec
    return {"copy_mib": copy_mib, "fetch_factor": ff, "write_factor": fw,
            "kernel_source_sha256": source_sha(), "kernels": out}


def write_md(summary, path: str, command: str, title: str):
    lines = [f"# {title}", "", "Commands (run from /tmp on the MI355X box, repository at $R):", "```",
             command, "```", "",
             f"Calibration: a device copy of {summary['copy_mib']} MiB in the same runs; "
             f"FETCH_SIZE factor {summary['fetch_factor']:.4f}, WRITE_SIZE factor "
             f"{summary['write_factor']:.4f} (known bytes / counter bytes).", "",
             "| kernel | dispatches | FETCH KiB / launch | WRITE KiB / launch | HBM bytes / launch (scaled) |",
             "|---|---:|---:|---:|---:|"]
    for fam, r in summary["kernels"].items():
        hb = r.get("hbm_bytes_per_launch")
        lines.append(f"| `{fam}` | {r['dispatches']} | {r['fetch_kib_per_launch'] or 0:.1f} | "
                     f"{r['write_kib_per_launch'] or 0:.1f} | {hb if hb is None else f'{hb:.4g}'} |")
    lines += ["", "Machine-readable (bench.py reads this block):", "```json",
              json.dumps(summary), "```", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def kernel_stats(path: str):
    """Per kernel: (calls, total ms, average us) from a rocprofv3 run, either
    its ``*_kernel_stats.csv`` (``--stats --output-format csv``) or its
    ``*_results.db`` (the default output of ``--kernel-trace``)."""
    rows = []
    if path.endswith(".csv"):
        for r in csv.DictReader(open(path)):
            rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]) / 1e6,
                         float(r["AverageNs"]) / 1e3))
    else:
        con = sqlite3.connect(path)
        q = ("select s.display_name, count(*), sum(k.duration), avg(k.duration) from kernels k "
             "join kernel_symbols s on k.kernel_id = s.kernel_id group by s.kernel_id")
        for name, calls, tot, avg in con.execute(q):
            rows.append((name, int(calls), tot / 1e6, avg / 1e3))
    merged = defaultdict(lambda: [0, 0.0])
    for name, calls, tot, _ in rows:
        k = short_name(name)
        merged[k][0] += calls
        merged[k][1] += tot
    out = [(k, c, t, t * 1e3 / c) for k, (c, t) in merged.items()]
    out.sort(key=lambda r: -r[2])
    return out


def write_trace_md(stats, path: str, command: str, title: str, notes: str = ""):
    total = sum(r[2] for r in stats) or 1.0
    lines = [f"# {title}", "", "Command (run from /tmp on the MI355X box, repository at $R):",
             "```", command, "```", ""]
    if notes:
        lines += [notes, ""]
    lines += ["| kernel | calls | total ms | avg us | % |", "|---|---:|---:|---:|---:|"]
    for k, c, t, a in stats:
        lines.append(f"| `{k}` | {c} | {t:.3f} | {a:.1f} | {100.0 * t / total:.2f} |")
    lines.append("")
    with open(path, "w") as f:
        f.write("\n".join(lines))


def valu_summary(path: str):
    """Per kernel family from a counter CSV of VALUBusy, SQ_INSTS_VALU and
    SQ_WAVES: dispatches, mean VALUBusy (percent of the time the CUs issue
    VALU instructions, rocprofv3's derived metric), and VALU instructions
    per wave (SQ_INSTS_VALU / SQ_WAVES summed over the dispatches)."""
    vals = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(path)):
        if not _family(r["Kernel_Name"]):
            continue
        vals[short_name(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out = {}
    for fam, c in vals.items():
        busy = c.get("VALUBusy", [])
        insts, waves = sum(c.get("SQ_INSTS_VALU", [])), sum(c.get("SQ_WAVES", []))
        out[fam] = {"dispatches": max(len(v) for v in c.values()),
                    "valu_busy_pct": sum(busy) / len(busy) if busy else None,
                    "valu_insts_per_wave": insts / waves if waves else None}
    return {"kernel_source_sha256": source_sha(), "kernels": out}


def write_valu_md(summary, path: str, command: str, title: str, notes: str = ""):
    lines = [f"# {title}", "", "Command (run from /tmp on the MI355X box, repository at $R):",
             "```", command, "```", ""]
    if notes:
        lines += [notes, ""]
    lines += ["| kernel | dispatches | VALUBusy % | VALU instructions per wave |",
              "|---|---:|---:|---:|"]
    for fam, r in sorted(summary["kernels"].items(), key=lambda kv: kv[0]):
        b, i = r["valu_busy_pct"], r["valu_insts_per_wave"]
        lines.append(f"| `{fam}` | {r['dispatches']} | {'' if b is None else f'{b:.1f}'} | "
                     f"{'' if i is None else f'{i:.0f}'} |")
    lines += ["", "Machine-readable:", "```json", json.dumps(summary), "```", ""]
    with open(path, "w") as f:
        f.write("\n".join(lines))


def load(path: str):
    """The summary stored in a profiles/*.md file, or None."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    i = text.find("```json")
    if i < 0:
        return None
    j = text.find("```", i + 7)
    return json.loads(text[i + 7:j])


if __name__ == "__main__":
    if sys.argv[1] == "valu":
        # python -m paper_2609_29554_amd.pmc valu COUNTERS.csv OUT.md "command" "title" ["notes"]
        sm = valu_summary(sys.argv[2])
        write_valu_md(sm, sys.argv[3], sys.argv[4], sys.argv[5],
                      sys.argv[6] if len(sys.argv) > 6 else "")
        print(json.dumps(sm, indent=1))
        sys.exit(0)
    if sys.argv[1] == "trace":
        # python -m paper_2609_29554_amd.pmc trace STATS OUT.md "command" "title" ["notes"]
        st = kernel_stats(sys.argv[2])
        write_trace_md(st, sys.argv[3], sys.argv[4], sys.argv[5],
                       sys.argv[6] if len(sys.argv) > 6 else "")
        for r in st[:12]:
            print(r)
        sys.exit(0)
    fetch_csv, write_csv, mib, out_md, cmd = sys.argv[1:6]
    title = sys.argv[6] if len(sys.argv) > 6 else "HBM traffic per kernel (rocprofv3 FETCH_SIZE / WRITE_SIZE)"
    s = summarize(fetch_csv, write_csv, float(mib))
    write_md(s, out_md, cmd, title)
    print(json.dumps(s, indent=1))
