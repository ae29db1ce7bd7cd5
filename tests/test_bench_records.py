"""The committed bench lines (profiles/bench_*.json) keep the bench output contract: the
headline fields, a roofline object whose fraction is achieved / peak at the peak of the
dominant kernel's own arithmetic, and, on the default line, the oracle's CPU baseline and the
counter-measured traffic."""
import glob
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RECORDS = sorted(glob.glob(os.path.join(ROOT, "profiles", "bench_*.json")))
PEAKS = {("mfma", "TFLOP/s"): (78.6, 157.3), ("hbm", "GB/s"): (8000.0,)}


def load(path):
    lines = [l for l in open(path).read().splitlines() if l.startswith("{")]
    assert len(lines) == 1, path
    return json.loads(lines[0])


def test_records_exist():
    names = {os.path.basename(p) for p in RECORDS}
    assert "bench_water4096_fp64.json" in names and "bench_water4096_fp32.json" in names


@pytest.mark.parametrize("path", RECORDS, ids=[os.path.basename(p) for p in RECORDS])
def test_contract_fields(path):
    d = load(path)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["higher_is_better"] is True and d["data"] == "synthetic"
    assert d["unit"] == "SCF steps/s" and d["value"] > 0
    assert abs(d["value"] * d["ms_per_step"] / 1e3 - 1.0) < 1e-3         # value = 1 / step time
    assert "workload" in d["config"] and "model" not in d["config"]
    assert d["dtype"] in ("f64", "f32+f64", "f32")
    r = d["roofline"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in r, k
    assert r["peak"] in PEAKS[(r["bound"], r["unit"])]
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-3
    if r["kernel"] == "ortho_update":                                    # FP64 in both forms
        assert r["peak"] == 78.6


def test_default_line_has_baseline_and_traffic():
    """The default line carries the oracle baseline; it carries the counter-measured traffic
    whenever it was taken on the kernel sources the counters were taken on."""
    d = load(os.path.join(ROOT, "profiles", "bench_water4096_fp64.json"))
    cpu = d["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["cores"] >= 1 and cpu["value"] > 0 and cpu["sample"]
    traffic = json.load(open(os.path.join(ROOT, "profiles", "traffic_water4096_fp64.json")))
    assert traffic["class_kernel"][d["roofline"]["kernel"]] in traffic["kernels"]
    if d.get("kernel_source_sha256") == traffic["kernel_source_sha256"]:
        assert d["roofline"]["traffic"] is not None
    else:
        assert d["roofline"]["traffic"] is None
