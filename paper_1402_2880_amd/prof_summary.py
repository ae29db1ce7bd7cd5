"""Short text summaries of rocprofv3 output for the profiles folder.

  python -m paper_1402_2880_amd.prof_summary kernels <stats.csv> <title> <command> > summary.md
  python -m paper_1402_2880_amd.prof_summary traffic <fetch.csv> <write.csv> <copy_mib> <title> <out.json>
                                                     <fetch command> <write command>
  python -m paper_1402_2880_amd.prof_summary l2 <tcc.csv> <title> <command> > summary.md

`kernels` turns a `--kernel-trace --stats` kernel_stats.csv into a table (calls, total, share,
average, min, max).  `traffic` takes two `--pmc` runs (FETCH_SIZE, WRITE_SIZE; counter_collection.csv)
of a program that first copied copy_mib MiB three times (bench.py --copy-calibration), scales each
counter by what it reads for those copies (a copy reads and writes copy_mib MiB), and writes per
kernel the mean HBM bytes per dispatch as JSON and Markdown; the JSON records the SHA-256 of the
kernel source so that a reader can tell whether the kernels have changed since.  `l2` takes one
`--pmc TCC_HIT_sum TCC_MISS_sum` run and tabulates the L2 hits, misses and hit rate per dispatch."""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("sscf_kernels.hip", "sscf_internal.h")]
# the library's kernel of each class of sscf_get_kernel_stats (the FP64 form at W = 96)
CLASS_KERNEL = {"spmm_tiles": "sscf::k_spmm_row<6, double>", "pair_overlap": "sscf::k_pair<3, 3>",
                "pair_fock": "sscf::k_pair<2, 2>", "ortho_update": "sscf::k_ortho_update<6>",
                "rotations": "sscf::k_givens_rb<6, double>"}


def source_sha256() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()


def short_name(name: str) -> str:
    """Kernel name without its argument list (templates kept)."""
    depth = 0
    for k, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:k].replace("void ", "").strip()
    return name.replace("void ", "").strip()


def kernels_table(stats_csv: str, title: str, command: str) -> str:
    rows = list(csv.DictReader(open(stats_csv)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"# rocprofv3 kernel summary: {title}", "", "Command (REPO = repository root on the GPU box):", "",
           f"    {command}", "", f"Kernel sources sha256 `{source_sha256()}`.", "",
           "Durations in microseconds; share of the summed kernel time; every launch of the run.", "",
           "| kernel | calls | total ms | share | avg us | min us | max us |", "|---|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:25]:
        t = float(r["TotalDurationNs"])
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {t / 1e6:.2f} | {100 * t / tot:.1f}% | "
                   f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} |")
    return "\n".join(out) + "\n"


def per_dispatch(counter_csv: str, counter: str):
    """{dispatch id: (kernel name, summed counter value)}"""
    acc = {}
    for r in csv.DictReader(open(counter_csv)):
        if r["Counter_Name"] != counter:
            continue
        d = r["Dispatch_Id"]
        name, v = acc.get(d, (short_name(r["Kernel_Name"]), 0.0))
        acc[d] = (name, v + float(r["Counter_Value"]))
    return acc


def traffic(fetch_csv: str, write_csv: str, copy_mib: float, title: str, out_json: str, cmd_f: str, cmd_w: str):
    f, w = per_dispatch(fetch_csv, "FETCH_SIZE"), per_dispatch(write_csv, "WRITE_SIZE")
    copy_kib = copy_mib * 1024.0

    def calib(acc):
        # the three calibration copies: the largest copy-kernel dispatches of the run
        vals = sorted((v for n, v in acc.values() if "copy" in n.lower()), reverse=True)[:3]
        if len(vals) < 3:
            raise RuntimeError("no calibration copies found")
        return vals, copy_kib / (sum(vals) / len(vals))

    fv, fs = calib(f)
    wv, ws = calib(w)
    per = defaultdict(lambda: [0, 0.0, 0, 0.0])
    for name, v in f.values():
        per[name][0] += 1
        per[name][1] += v
    for name, v in w.values():
        per[name][2] += 1
        per[name][3] += v
    kern = {}
    for name, (nf, sf, nw, sw) in per.items():
        if not name.startswith("sscf::") or nf == 0 or nw == 0:
            continue
        fm, wm = sf / nf, sw / nw
        kern[name] = dict(dispatches=nf, fetch_kib_mean=fm, write_kib_mean=wm,
                          hbm_bytes_per_launch=(fm * fs + wm * ws) * 1024.0)
    rec = dict(workload=title, kernel_source_sha256=source_sha256(), commands=[cmd_f, cmd_w],
               calibration=dict(copy_kib_read_and_written=copy_kib, fetch_size_kib_read=fv, write_size_kib_read=wv,
                                fetch_scale=fs, write_scale=ws),
               class_kernel=CLASS_KERNEL,
               kernels=dict(sorted(kern.items(), key=lambda kv: -kv[1]["hbm_bytes_per_launch"])))
    json.dump(rec, open(out_json, "w"), indent=1)
    md = [f"# HBM traffic per launch: {title}", "", "Two rocprofv3 counter runs (one counter each), REPO = "
          "repository root on the GPU box:", "", f"    {cmd_f}", f"    {cmd_w}", "",
          f"Kernel sources sha256 `{rec['kernel_source_sha256']}`.", "",
          f"Scale: a {copy_mib:g} MiB device copy ({copy_kib:,.0f} KiB read and written) reads FETCH_SIZE "
          f"{sum(fv) / 3:,.0f} KiB and WRITE_SIZE {sum(wv) / 3:,.0f} KiB, so FETCH_SIZE is multiplied by {fs:.3f} "
          f"and WRITE_SIZE by {ws:.3f}.", "", "Means over the dispatches of the run:", "",
          "| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM GB per launch (scaled) |", "|---|---|---|---|---|"]
    for name, k in rec["kernels"].items():
        md.append(f"| `{name}` | {k['dispatches']} | {k['fetch_kib_mean']:.0f} | {k['write_kib_mean']:.0f} | "
                  f"{k['hbm_bytes_per_launch'] / 1e9:.3f} |")
    open(os.path.splitext(out_json)[0] + ".md", "w").write("\n".join(md) + "\n")


def l2_table(tcc_csv: str, title: str, command: str) -> str:
    hits, miss = per_dispatch(tcc_csv, "TCC_HIT_sum"), per_dispatch(tcc_csv, "TCC_MISS_sum")
    per = defaultdict(lambda: [0, 0.0, 0.0])
    for d, (name, h) in hits.items():
        if d in miss:
            per[name][0] += 1
            per[name][1] += h
            per[name][2] += miss[d][1]
    rows = sorted(per.items(), key=lambda kv: -(kv[1][1] + kv[1][2]) / kv[1][0])[:12]
    out = [f"# L2 (TCC) hits and misses per dispatch: {title}", "", "One rocprofv3 counter run (REPO = repository "
           "root on the GPU box):", "", f"    {command}", "", f"Kernel sources sha256 `{source_sha256()}`.", "",
           "Means over the dispatches of the run; a miss goes to the fabric (MALL or HBM).", "",
           "| kernel | dispatches | hits | misses | hit rate |", "|---|---|---|---|---|"]
    for name, (n, h, m) in rows:
        out.append(f"| `{name}` | {n} | {h / n:,.0f} | {m / n:,.0f} | {h / max(h + m, 1.0):.3f} |")
    return "\n".join(out) + "\n"


if __name__ == "__main__":
    if sys.argv[1] == "kernels":
        sys.stdout.write(kernels_table(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif sys.argv[1] == "l2":
        sys.stdout.write(l2_table(sys.argv[2], sys.argv[3], sys.argv[4]))
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], float(sys.argv[4]), sys.argv[5], sys.argv[6], sys.argv[7], sys.argv[8])
    else:
        raise SystemExit(__doc__)
