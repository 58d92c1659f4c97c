"""Host logic of the benchmark (CPU): the work model behind the roofline figure, the reading of
rocprofv3 output (kernel names, the timed-region filter, CSV dispatch records), and the lookup
of committed counter results."""

import json
import math
import os

import pytest

import bench


def test_flop_model_examples():
    # the worked example of the design notes: N = 256, C = 2, overlap 256
    assert bench.flops_per_eval(256, 2, 256, False) == pytest.approx(1.14e5, rel=0.01)
    assert bench.flops_per_eval(256, 2, 256, True) == pytest.approx(3.48e5, rel=0.01)
    # the pieces: slow series per sample (+10 with T), one DFT per channel, 20 per bin and channel
    N, C, ov = 512, 3, 700
    f = bench.flops_per_eval(N, C, ov, False)
    assert f == 334 * N + C * 5 * N * math.log2(N) + 20 * C * ov
    g = bench.flops_per_eval(N, C, ov, True)
    assert g - f == C * 5 * N * math.log2(N) + 825 * N + 6 * C * ov
    assert bench.sincos_per_eval(N, False) == 4 * N and bench.sincos_per_eval(N, True) == 8 * N


def test_kernel_key():
    assert bench._kernel_key("void gbx::k_batch<double, 512, 128, 3, 4, 1, 1>(gbx::BatchArgs)") == \
        "k_batch<double,512,128,3,4,1,1>"
    assert bench._kernel_key("k_mh_chain(gbx::ChainWin const*)") == "k_mh_chain"


def _bench_line(kern, n, region):
    return {"roofline": {"kernel": kern, "launches_in_region": n}, "timed_region_ns": region}


def test_timed_region_filter():
    k = "k_batch<float,512,64,3,4,2,1>"
    disp = [(k, 100, 200, None), (k, 300, 400, None), (k, 500, 600, None), ("other", 150, 160, None),
            (k, 1100, 1200, None), (k, 1300, 1400, None)]
    # the first clock's window holds 3 launches (wrong count), the second's exactly 2
    line = _bench_line(k, 2, {"monotonic": [50, 650], "boottime": [1050, 1450]})
    sel = bench._in_region(disp, line)
    assert [d[1] for d in sel] == [1100, 1300]
    with pytest.raises(ValueError):
        bench._in_region(disp, _bench_line(k, 5, {"monotonic": [50, 650]}))


def test_dispatches_from_csv(tmp_path):
    run = tmp_path / "run" / "host"
    run.mkdir(parents=True)
    (run / "x_kernel_trace.csv").write_text(
        "Kernel_Name,Start_Timestamp,End_Timestamp\n"
        "\"void gbx::k_batch<float, 64, 16, 2, 4, 1, 2>(gbx::BatchArgs)\",10,20\n"
        "k_mh_chain(gbx::ChainWin const*),30,40\n")
    d = bench._dispatches(str(tmp_path / "run"))
    assert d == [("k_batch<float,64,16,2,4,1,2>", 10, 20, None), ("k_mh_chain", 30, 40, None)]
    with pytest.raises(FileNotFoundError):
        bench._dispatches(str(tmp_path / "empty"))


def test_committed_traffic_lookup(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "hbm_traffic.txt").write_text(
        "# comment line kernel_src=x kernel=k bytes=1 evals=1\n"
        f"kernel_src={h} kernel=k_batch<float,512,64,3,4,2,1> evals=400000 bytes=80000000\n"
        f"kernel_src=0000 kernel=k_batch<float,256,32,2,4,2,2> evals=100 bytes=100\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    # exact kernel, scaled to the evaluations of a launch
    assert bench.committed_traffic("k_batch<float,512,64,3,4,2,1>", 200000) == 40000000.0
    # another register budget of the family is another kernel (its own machine code): none
    assert bench.committed_traffic("k_batch<float,512,64,3,4,2,2>", 400000) is None
    # another family, or counters taken on other kernel sources: none
    assert bench.committed_traffic("k_batch<float,512,64,2,4,2,1>", 400000) is None
    assert bench.committed_traffic("k_batch<float,256,32,2,4,2,2>", 100) is None


def test_counter_summary(tmp_path):
    """Per-engine counter rows are summed per dispatch, only timed-region dispatches count, and
    the SIMD busy share is waves per SIMD times the per-wave VALU share."""
    k = "k_batch<float,512,64,3,4,2,1>"
    run = tmp_path / "pmc" / "host"
    run.mkdir(parents=True)
    rows = ["Kernel_Name,Start_Timestamp,End_Timestamp,Counter_Name,Counter_Value"]
    name = f"\"void gbx::{k.replace(',', ', ')}(gbx::BatchArgs)\""
    # one dispatch before the region, two inside; each counter split over two engine rows
    for t0, t1 in ((100, 200), (1_000_000, 5_000_000), (6_000_000, 12_000_000)):
        per = {"SQ_WAVES": 2048, "SQ_WAVE_CYCLES": 1000.0, "SQ_BUSY_CYCLES": 1.0, "SQ_WAIT_ANY": 250.0,
               "SQ_WAIT_INST_ANY": 1.0, "SQ_ACTIVE_INST_ANY": 1.0, "SQ_ACTIVE_INST_VALU": 400.0,
               "SQ_INSTS_VALU": 200.0}
        if t0 == 100:
            per["SQ_ACTIVE_INST_VALU"] = 0.0
        for c, v in per.items():
            rows += [f"{name},{t0},{t1},{c},{v / 2}"] * 2
    (run / "x_counter_collection.csv").write_text("\n".join(rows) + "\n")
    bj = tmp_path / "b.json"
    bj.write_text(json.dumps({"roofline": {"kernel": k, "launches_in_region": 2},
                              "timed_region_ns": {"monotonic": [900, 13_000_000]}}) + "\n")
    out = bench.counter_summary(str(bj), str(tmp_path / "pmc")).splitlines()
    assert len(out) == 2 and out[1].split()[0] == k
    f = out[1].split()
    assert f[1] == "2" and float(f[2]) == pytest.approx(5.0)      # dispatches, avg ms
    assert float(f[3]) == pytest.approx(2.0)                         # 2048 waves / 1024 SIMDs
    assert float(f[4]) == pytest.approx(0.4) and float(f[5]) == pytest.approx(0.25)
    assert float(f[6]) == pytest.approx(0.8) and float(f[7]) == pytest.approx(2.0)
