"""Host-side checks of the rocprofv3 summary tool and of bench.py's lookup of the measured
traffic (synthetic CSV files in the layout rocprofv3 writes; no GPU)."""
import csv
import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_counter_values_in_dispatch_order(tmp_path):
    from paper_2501_03759_amd import profiling
    rows = [[7, "FETCH_SIZE", "void lbch::batch_step<float, 128, true, 2>", 30.0],
            [2, "FETCH_SIZE", "void lbch::batch_step<float, 64, true, 1>", 10.0],
            [5, "WRITE_SIZE", "void lbch::batch_step<float, 128, true, 2>", 99.0],
            [4, "FETCH_SIZE", "lbch::copy16_k", 5.0],
            [3, "FETCH_SIZE", "void lbch::batch_step<float, 128, true, 2>", 20.0]]
    _write_csv(str(tmp_path / "r" / "run_counter_collection.csv"),
               ["Dispatch_Id", "Counter_Name", "Kernel_Name", "Counter_Value"], rows)
    assert profiling.counter_values(str(tmp_path / "r"), "FETCH_SIZE", "batch_step") == [10.0, 20.0, 30.0]
    assert profiling.counter_values(str(tmp_path / "r"), "FETCH_SIZE", "copy16_k") == [5.0]


def test_last_dispatches_are_one_kernel(tmp_path):
    from paper_2501_03759_amd import profiling
    a, b = "void lbch::batch_step<float, 256, true, 2>(x)", "void lbch::batch_step<float, 128, true, 2>(x)"
    rows = [[a, 100, 150], [b, 300, 310], [b, 200, 230], [b, 400, 440], ["lbch::copy16_k", 500, 900]]
    _write_csv(str(tmp_path / "t" / "run_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"],
               rows)
    name, durs = profiling.last_dispatches(str(tmp_path / "t"), "batch_step", 3)
    assert name == b and durs == [30, 10, 40]                       # in start order
    with pytest.raises(ValueError):
        profiling.last_dispatches(str(tmp_path / "t"), "batch_step", 4)


def test_measured_traffic_requires_matching_source_size_depth_and_shape(tmp_path):
    sys.path.insert(0, ROOT)
    import bench
    from paper_2501_03759_amd.profiling import kernel_hash
    rec = {"kernel_sha256_16": kernel_hash("d2q9"), "nodes": 1000, "precision": "fp32", "depth": 2,
           "tiling": [128, 32], "bytes_per_launch": 123.0}
    p = str(tmp_path / "prof.json")
    json.dump(rec, open(p, "w"))
    assert bench.measured_traffic(1000, "fp32", 2, path=p, tiling=(128, 32)) == 123.0
    assert bench.measured_traffic(1000, "fp32", 2, path=p) == 123.0
    assert bench.measured_traffic(1000, "fp32", 2, path=p, tiling=(128, 64)) is None
    assert bench.measured_traffic(999, "fp32", 2, path=p, tiling=(128, 32)) is None
    assert bench.measured_traffic(1000, "fp32", 1, path=p, tiling=(128, 32)) is None
    assert bench.measured_traffic(1000, "fp64", 2, path=p, tiling=(128, 32)) is None
    json.dump(dict(rec, kernel_sha256_16="0" * 16), open(p, "w"))
    assert bench.measured_traffic(1000, "fp32", 2, path=p, tiling=(128, 32)) is None
    assert bench.measured_traffic(1000, "fp32", 2, path=str(tmp_path / "missing.json")) is None


def test_unet_layer_table_from_a_synthetic_trace(tmp_path):
    # three forward passes of a 2-level net (6 convolutions each) and one weight-gradient
    # dispatch after them; the first pass is dropped as a warm-up, the training step's
    # forward convolutions after the weight gradient are not counted
    from paper_2501_03759_amd import profiling
    layers = profiling.unet_layers((32, 64), 5, 2, 32)
    assert [l[0] for l in layers] == ["enc0a", "enc0b", "enc1a", "enc1b", "dec0a", "dec0b"]
    rows, t = [], 0
    for g in range(3):
        rows.append(["lbch::pack_input_k", t, t + 5])
        t += 10
        for i in range(6):
            dur = 1000 * (i + 1) * (2 if g == 0 else 1)
            name = "void lbsg::conv3_first_k<64>" if i == 0 else "void lbsg::conv3_fwd_k<32, true, false>"
            rows.append([name, t, t + dur])
            t += dur + 10
    rows.append(["void lbsg::conv3_dw_k<64>", t, t + 100])
    t += 200
    # after the training step: two inference passes (the first a warm-up)
    for g in range(2):
        for i in range(6):
            dur = 3000 * (i + 1) * (2 if g == 0 else 1)
            name = "void lbsg::conv3_first_k<64>" if i == 0 else "void lbsg::conv3_fwd_k<32, true, false>"
            rows.append([name, t, t + dur])
            t += dur + 10
    _write_csv(str(tmp_path / "tr" / "run_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    table = profiling.unet_profile(str(tmp_path / "tr"), [], (32, 64), 5, 2, 32)
    assert [round(r["us"], 3) for r in table] == [1.0, 2.0, 3.0, 4.0, 5.0, 6.0]
    r0 = table[0]
    assert r0["gflop"] == 18.0 * 2 * 32 * 32 * 5 * 32 / 1e9
    # the first layer's algorithmic bytes: its 5 real input channels and 32 output channels, BF16
    assert r0["ai"] == r0["gflop"] * 1e9 / (2 * 2 * 32 * 32 * (5 + 32))
    assert r0["roofline_tflops"] == min(2500.0, r0["ai"] * 8.0)
    inf = profiling.unet_profile(str(tmp_path / "tr"), [], (32, 64), 5, 2, 32, after_training=True)
    assert [round(r["us"], 3) for r in inf] == [3.0, 6.0, 9.0, 12.0, 15.0, 18.0]


def test_unet_inference_table_with_the_fused_first_block(tmp_path):
    # inference passes whose first block is one launch (conv3_pair0_k): one row for both
    # convolutions, with the block's input and outputs as its bytes (no intermediate)
    from paper_2501_03759_amd import profiling
    rows, t = [], 0
    rows.append(["void lbsg::conv3_dw_k<64>", t, t + 100])
    t += 200
    for g in range(3):
        names = ["lbsg::conv3_pair0_k<4>"] + ["void lbsg::conv3_fwd_k<32, true, false>"] * 4
        for i, name in enumerate(names):
            dur = 1000 * (i + 1)
            rows.append([name, t, t + dur])
            t += dur + 10
    _write_csv(str(tmp_path / "tr" / "run_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    table = profiling.unet_profile(str(tmp_path / "tr"), [], (32, 64), 5, 1, 64, after_training=True)
    assert [r["layer"] for r in table] == ["enc0a+b", "enc1a", "enc1b", "dec0a", "dec0b"]
    assert [round(r["us"], 3) for r in table] == [1.0, 2.0, 3.0, 4.0, 5.0]
    px = 64 * 64
    assert table[0]["gflop"] == 18.0 * px * (5 * 32 + 32 * 32) / 1e9
    assert table[0]["alg_bytes"] == 2 * px * (5 + 32) + 2 * (px // 4) * 32


def test_unet_table_shows_valu_busy_beside_mfma_util(tmp_path):
    # a --pmc run with MfmaUtil and VALUBusy per dispatch: the table takes the mean over the
    # passes after the warm-up, per layer, and prints a VALUBusy column only when collected
    from paper_2501_03759_amd import profiling
    rows, ctr, t, did = [], [], 0, 0
    for g in range(3):
        for i in range(6):
            name = "void lbsg::conv3_first_k<64>" if i == 0 else "void lbsg::conv3_fwd_k<32, true, false>"
            rows.append([name, t, t + 1000])
            t += 1010
            did += 1
            ctr.append([did, name, "MfmaUtil", 10.0 * (i + 1) + g])
            ctr.append([did, name, "VALUBusy", 80.0 - i + g])
    _write_csv(str(tmp_path / "tr" / "run_kernel_trace.csv"), ["Kernel_Name", "Start_Timestamp", "End_Timestamp"], rows)
    _write_csv(str(tmp_path / "pmc" / "run_counter_collection.csv"),
               ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], ctr)
    table = profiling.unet_profile(str(tmp_path / "tr"), [str(tmp_path / "pmc")], (32, 64), 5, 2, 32)
    assert [r["mfma_util_pct"] for r in table] == [10.0 * (i + 1) + 1.5 for i in range(6)]
    assert [r["valu_busy_pct"] for r in table] == [80.0 - i + 1.5 for i in range(6)]
    lines = profiling.unet_lines(table)
    assert lines[0].endswith("| MfmaUtil % | VALUBusy % |") and lines[2].endswith("| 11.5 | 81.5 |")
    plain = profiling.unet_lines([{k: v for k, v in r.items() if k != "valu_busy_pct"} for r in table])
    assert plain[0].endswith("| MfmaUtil % |") and "VALUBusy" not in "".join(plain)
