"""Host-side tools without a GPU: the rocprofv3 CSV summaries, and the bench
script's traffic lookup and one-GPU guard."""
import csv
import json
import os
import statistics
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2408_03452_amd import tracesum  # noqa: E402


def _write_trace(path, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        t = 0
        for name, grid, dur_ns in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Start_Timestamp": t,
                        "End_Timestamp": t + dur_ns})
            t += dur_ns + 1000


def test_split_separates_workloads_that_share_a_launch_size():
    fast = [20.0 + 0.01 * i for i in range(300)]
    slow = [110.0 + 0.01 * i for i in range(1000)]
    parts = tracesum._split(fast + slow)
    assert [label for label, _ in parts] == [" (fast)", " (slow)"]
    assert len(parts[0][1]) == 300 and len(parts[1][1]) == 1000
    # one workload, spread within 2x: one row
    assert len(tracesum._split([100.0 + i for i in range(50)])) == 1
    # a handful of outliers (< 1 % of the calls) do not make a row of their own
    assert len(tracesum._split([110.0] * 1000 + [5.0] * 3)) == 1
    # launches in between (cold starts, early exits) do not hide two workloads
    mixed = fast + slow + [30.0 + 10 * i for i in range(8)] + [3.0] * 5
    parts = tracesum._split(mixed)
    assert len(parts) == 2
    assert abs(statistics.median(parts[1][1]) - statistics.median(slow)) < 1.0
    assert abs(statistics.median(parts[0][1]) - statistics.median(fast)) < 1.0


def test_trace_summary_rows(tmp_path, capsys):
    rows = [("void stencil_v4<1>(mffv::Geom)", 524288, 110_000)] * 200
    rows += [("void stencil_v4<1>(mffv::Geom)", 524288, 19_000)] * 100
    rows += [("mffv::(anonymous namespace)::phase_b", 262144, 33_000)] * 50
    _write_trace(tmp_path / "x_kernel_trace.csv", rows)
    tracesum.trace(str(tmp_path))
    out = capsys.readouterr().out
    lines = [l for l in out.splitlines() if l.startswith("| `")]
    assert any("stencil_v4<1> (slow)` | 524288 | 200 | 22.00 | 110.00 | 110.00" in l for l in lines)
    assert any("stencil_v4<1> (fast)` | 524288 | 100 | 1.90 | 19.00 | 19.00" in l for l in lines)
    assert any("`phase_b` | 262144 | 50 |" in l for l in lines)


def test_pmc_summary_skips_idle_dispatches(tmp_path, capsys):
    with open(tmp_path / "p_counter_collection.csv", "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for v in [1000.0] * 4 + [2.0] * 2:
            w.writerow({"Kernel_Name": "copy_probe", "Grid_Size": 4096, "Counter_Name": "FETCH_SIZE",
                        "Counter_Value": v})
    tracesum.pmc(str(tmp_path))
    out = capsys.readouterr().out
    assert "| `copy_probe` | 4096 | FETCH_SIZE | 4 | 1000.0 | 2 |" in out


def test_bench_traffic_lookup():
    import bench
    t = {"profile": "p", "by_launch": [({"ci": 8, "remap": 0, "seg": -1}, 111), ({"ci": 16, "remap": 1, "seg": -1}, 222)]}
    assert bench.traffic_for(t, {"ci": 16, "remap": 1, "seg": -1, "vec": 4}) == 222
    assert bench.traffic_for(t, {"ci": 16, "remap": 0, "seg": -1, "vec": 4}) is None
    assert bench.traffic_for(None, {"ci": 8, "remap": 0, "seg": -1}) is None
    # every measured shape is distinct, and each figure is above the kernel's algorithmic bytes
    shapes = [json.dumps(l, sort_keys=True) for l, _ in bench.TRAFFIC["two_phase"]["by_launch"]]
    assert len(set(shapes)) == len(shapes)
    alg = bench.PHASE_A_BYTES_PER_CELL * 256 ** 3
    assert all(alg < b < 1.5 * alg for _, b in bench.TRAFFIC["two_phase"]["by_launch"])


def test_bench_refuses_more_than_one_gpu():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode != 0
    assert "one GPU" in (res.stdout + res.stderr)


def test_bench_phase_a_byte_model():
    """Phase A moves 24 B/cell at k = 0 (r, faces in; p, q out), 28 on odd k
    (also p_{k-1} in) and 40 on even k >= 2 (also x and p_{k-2} in, x out)."""
    import bench
    assert [bench.phase_a_bytes(k) for k in range(5)] == [24, 28, 40, 28, 40]
    assert bench.phase_a_bytes_mean(32) == 33.5
    assert bench.phase_a_bytes_mean(64) == 33.75
    assert bench.PHASE_A_BYTES_PER_CELL == (28 + 40) / 2
    assert bench.CG_BYTES_PER_CELL_ITER == bench.PHASE_A_BYTES_PER_CELL + bench.PHASE_B_BYTES_PER_CELL


def test_stream_mixes_match_the_byte_model():
    """Each kernel's mix of FP32 arrays read / written, streamed by the probe,
    moves the kernel's algorithmic bytes per cell: apply 20, phase A 28 (odd k)
    and 40 (even k), phase B 12."""
    import bench
    m = bench.STREAM_MIXES
    assert 4 * sum(m["apply"]) == bench.APPLY_BYTES_PER_CELL
    assert 4 * sum(m["phase_a_odd"]) == bench.phase_a_bytes(1)
    assert 4 * sum(m["phase_a_even"]) == bench.phase_a_bytes(2)
    assert 4 * sum(m["phase_b"]) == bench.PHASE_B_BYTES_PER_CELL
    # writes: apply y; phase A p, q (+ x on even k); phase B r
    assert [m[k][1] for k in ("apply", "phase_a_odd", "phase_a_even", "phase_b")] == [1, 2, 3, 1]
    # face-list apply: 12 B per cell and 16 B per face
    assert bench.face_apply_bytes(10, 3) == 12 * 10 + 16 * 3
