"""Host logic of bench.py that needs no GPU: the committed counter summaries
parse, are consistent with the workload they describe, and are matched to a
run only in the exact launch shape they were taken on."""
import os

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def fields(path):
    return bench._summary_fields(path)


def test_counter_summaries_parse_and_are_consistent():
    kv = fields(bench.COUNTERS_FILE)
    shape = tuple(int(v) for v in kv["launch"].split(","))
    assert len(shape) == 3 and shape[2] in (3, 4)  # a multi-step variant
    state = float(kv["state_bytes_per_launch"])
    assert state == 72.0 * 8192 * 8192  # the stored state (9 FP32 planes) read and written once per launch
    hbm = float(kv["hbm_bytes_per_launch"])
    assert state <= hbm <= 2.0 * state  # writes are exact; reads add halo rows and columns
    sq = fields(bench.SQ_FILE)
    assert sq["launch"] == kv["launch"] and sq["kernel_source_sha"] == kv["kernel_source_sha"]
    assert float(sq["valu_instructions_per_launch"]) > 0 and float(sq["launch_us"]) > 0
    # FP32 operations: 64 lanes x (ADD + MUL + TRANS + 2 FMA) wave instructions
    w = {k: float(sq[k]) for k in ("SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_TRANS_F32",
                                     "SQ_INSTS_VALU_FMA_F32")}
    flops = 64 * (w["SQ_INSTS_VALU_ADD_F32"] + w["SQ_INSTS_VALU_MUL_F32"] + w["SQ_INSTS_VALU_TRANS_F32"]
                  + 2 * w["SQ_INSTS_VALU_FMA_F32"])
    assert float(sq["fp32_flops_per_launch"]) == pytest.approx(flops, rel=1e-9)


def test_counters_are_matched_on_the_full_launch_shape():
    kv = fields(bench.COUNTERS_FILE)
    shape = tuple(int(v) for v in kv["launch"].split(","))
    if kv.get("kernel_source_sha") != bench.kernel_source_hash():
        pytest.skip("the committed counters were taken on other kernel sources")
    assert bench.profiled_launch() == shape
    assert bench.measured_traffic(shape) == float(kv["hbm_bytes_per_launch"])
    other_strip = (shape[0], shape[1] + 8, shape[2])
    assert bench.measured_traffic(other_strip) is None
    assert bench.measured_valu_instructions((shape[0] + 32, shape[1], shape[2])) is None
    assert bench.measured_traffic(None) is None


def test_trace_summary_names_the_profiled_launch():
    kv = fields(bench.COUNTERS_FILE)
    text = open(os.path.join(ROOT, "profiles", "step_f32_8192_kernel_trace.md")).read()
    assert "--launch " + kv["launch"] in text
    assert "stepS_kernel_lds<0, %s, 3, 0>" % kv["launch"].split(",")[0] in text


def test_multi_gpu_request_is_refused():
    import subprocess
    import sys

    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
