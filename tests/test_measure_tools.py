"""Host logic of the measurement tools (no GPU): the HBM-traffic summary of
rocprofv3 counter collections, and the bench's accounting of the fused
latent kernel."""
import csv
import json
import os

import pytest

import bench
from paper_2305_11566_amd import profile_traffic as pt

KIB = 1024.0


def _write_counters(d, rows):
    """rows: [(kernel name, KiB)] in dispatch order -> one counter_collection.csv."""
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "pmc_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Value"])
        w.writeheader()
        for i, (n, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": n, "Counter_Value": v})


def _dispatches():
    """Census, cost, one forward with every layer launched (E3 and G2 split,
    each followed by its sum), one inference forward with the fused kernel,
    then the 64 MiB copy."""
    conv = "void sv::k_conv<0, 3, 2, 2, 32, 2, 2>(sv::ConvParams)"
    red = "void sv::k_conv_split_reduce<0>(sv::ConvParams, int)"
    lat = "void sv::k_latent<0>(sv::ConvParams, sv::ConvParams, int)"
    fin = "void sv::k_final<0>(float const*, int)"
    seq = [("void sv::k_reduce_census<4, 4>(unsigned char const*)", 10.0),
           ("void sv::k_cost_wta<4>(unsigned long const*)", 2.0)]
    unf = [(conv, 1.0), (conv, 2.0), (conv, 3.0), (red, 0.5), (conv, 4.0), (conv, 5.0),
           (conv, 6.0), (red, 0.25), (conv, 7.0), (conv, 8.0), (fin, 9.0)]
    fus = [(conv, 11.0), (conv, 12.0), (conv, 13.0), (lat, 14.0), (conv, 15.0), (conv, 16.0),
           (conv, 17.0), (fin, 18.0)]
    copy = [("__amd_rocclr_copyBuffer", 2.0 * 65536.0)]  # FETCH reads twice the copy's bytes
    return seq + unf + fus + copy


def test_traffic_summary_fused_and_split(tmp_path):
    rows = _dispatches()
    _write_counters(tmp_path / "tf", rows)
    _write_counters(tmp_path / "tw", [(n, v if "copyBuffer" not in n else 65536.0) for n, v in rows])
    cfgs = ["c%d" % i for i in range(9)]
    dflt = ["d%d" % i for i in range(9)]
    (tmp_path / "names.json").write_text(json.dumps([cfgs, dflt]))
    out = tmp_path / "traffic.json"
    pt.summarize(str(tmp_path / "tf"), str(tmp_path / "tw"), str(tmp_path / "names.json"), str(out))
    doc = json.loads(out.read_text())
    assert doc["counter_scale"]["FETCH_SIZE"] == pytest.approx(0.5)
    assert doc["counter_scale"]["WRITE_SIZE"] == pytest.approx(1.0)
    L = doc["layers"]
    key = "f32|B1|375x1242|{}|{}".format
    # each layer launched: a split layer carries its sum's bytes
    assert L[key("E3", "c2")]["write_bytes"] == round(3.5 * KIB)
    assert L[key("G2", "c5")]["write_bytes"] == round(6.25 * KIB)
    assert L[key("G3", "c4")]["write_bytes"] == round(5.0 * KIB)
    assert L[key("G0", "c7")]["fetch_bytes"] == round(0.5 * 8.0 * KIB)
    # the inference pass: head and G3 as one kernel, recorded as HEAD+G3
    assert L[key("HEAD+G3", "fused")]["write_bytes"] == round(14.0 * KIB)
    assert L[key("HEAD+G3", "fused")]["kernel"].endswith("k_latent<0>")
    assert L[key("G2", "d5")]["write_bytes"] == round(15.0 * KIB)
    assert key("HEAD", "d3") not in L and key("G3", "d4") not in L
    assert doc["final_gather"]["write_bytes"] == round(18.0 * KIB)
    assert doc["census"]["write_bytes"] == pytest.approx(10.0 * KIB)
    assert doc["source_hash"] == pt.source_hash()


def test_bench_merges_fused_latent_stage():
    prof = {"E3": (1.0, 5), "HEAD": (2.0, 5), "G3": (0.0, 0), "G2": (3.0, 5)}
    m = bench.merge_latent(prof)
    assert "HEAD" not in m and "G3" not in m and m["HEAD+G3"] == (2.0, 5)
    assert m["E3"] == (1.0, 5) and m["G2"] == (3.0, 5)
    # two launches: unchanged
    two = {"HEAD": (2.0, 5), "G3": (1.0, 5)}
    assert bench.merge_latent(two) == two


def test_bench_fused_latent_work_is_both_layers():
    for B in (1, 64):
        _, both, unit = bench.stage_work("HEAD+G3", B, "f32")
        _, head, _ = bench.stage_work("HEAD", B, "f32")
        _, g3, _ = bench.stage_work("G3", B, "f32")
        assert unit == "TFLOP" and both == pytest.approx(head + g3)
    # 468 latent pixels at batch 1: 2 x 468 x (256 x 128 + 128 x 128) FLOP
    assert bench.stage_work("HEAD+G3", 1, "f32")[1] == pytest.approx(2 * 468 * (256 * 128 + 128 * 128) / 1e12)
