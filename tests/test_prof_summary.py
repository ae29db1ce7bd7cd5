"""The profile summarizer (paper_1402_2880_amd/prof_summary.py) on small synthetic rocprofv3 CSVs:
the calibration of the HBM counters by the copy kernels, the per-dispatch means and the L2 rates."""
import csv
import json
import os

from paper_1402_2880_amd import prof_summary as ps


def write_counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


def test_short_name_drops_arguments_keeps_templates():
    assert ps.short_name("void sscf::k_pair<3, 3>(int, int const*)") == "sscf::k_pair<3, 3>"
    assert ps.short_name("sscf::k_fill(double*, unsigned long, double)") == "sscf::k_fill"


def test_traffic_scales_each_counter_by_the_copies(tmp_path):
    copy = "__amd_rocclr_copyBuffer"
    # three 512 MiB copies: FETCH_SIZE reads half of what was read, WRITE_SIZE all of it (split over
    # two counter instances of one dispatch, which are summed)
    fetch = [(1, copy, "FETCH_SIZE", 131072), (1, copy, "FETCH_SIZE", 131072), (2, copy, "FETCH_SIZE", 262144),
             (3, copy, "FETCH_SIZE", 262144), (4, "void sscf::k_a(int)", "FETCH_SIZE", 1000),
             (5, "void sscf::k_a(int)", "FETCH_SIZE", 3000), (6, "void other(int)", "FETCH_SIZE", 7)]
    write = [(1, copy, "WRITE_SIZE", 524288), (2, copy, "WRITE_SIZE", 524288), (3, copy, "WRITE_SIZE", 524288),
             (4, "void sscf::k_a(int)", "WRITE_SIZE", 500), (5, "void sscf::k_a(int)", "WRITE_SIZE", 1500),
             (6, "void other(int)", "WRITE_SIZE", 7)]
    fp, wp = str(tmp_path / "f.csv"), str(tmp_path / "w.csv")
    write_counters(fp, fetch)
    write_counters(wp, write)
    out = str(tmp_path / "t.json")
    ps.traffic(fp, wp, 512, "synthetic", out, "cmd f", "cmd w")
    rec = json.load(open(out))
    cal = rec["calibration"]
    assert abs(cal["fetch_scale"] - 2.0) < 1e-12 and abs(cal["write_scale"] - 1.0) < 1e-12
    assert list(rec["kernels"]) == ["sscf::k_a"]                    # only the library's kernels
    k = rec["kernels"]["sscf::k_a"]
    assert k["dispatches"] == 2 and k["fetch_kib_mean"] == 2000 and k["write_kib_mean"] == 1000
    assert abs(k["hbm_bytes_per_launch"] - (2000 * 2.0 + 1000 * 1.0) * 1024) < 1e-6
    assert rec["kernel_source_sha256"] == ps.source_sha256()
    assert os.path.exists(str(tmp_path / "t.md"))


def test_l2_table_rates(tmp_path):
    p = str(tmp_path / "tcc.csv")
    write_counters(p, [(1, "void sscf::k_a(int)", "TCC_HIT_sum", 30), (1, "void sscf::k_a(int)", "TCC_MISS_sum", 10),
                       (2, "void sscf::k_a(int)", "TCC_HIT_sum", 10), (2, "void sscf::k_a(int)", "TCC_MISS_sum", 10)])
    md = ps.l2_table(p, "synthetic", "cmd")
    row = [l for l in md.splitlines() if l.startswith("| `sscf::k_a`")][0]
    assert row == "| `sscf::k_a` | 2 | 20 | 10 | 0.667 |"
