"""CPU checks of the benchmark's host logic: the algorithmic byte model, the gating of the
measured HBM traffic on the kernel sources it was taken on, and the one-GPU guard."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_cavity_byte_model():
    b = load_bench()
    # the scope table's model per insertion: 44 + 64 W + 32 C + 16 F + 32 V, W = 4, V = 30;
    # at C = 20, F = 26 it is 2316 B
    assert b.cavity_bytes_per_insertion(20, 26) == 44 + 4 * 64 + 20 * 32 + 26 * 16 + 30 * 32 == 2316
    assert b.cavity_bytes_per_insertion(0, 0, W=0, V=0) == 44
    assert b.cavity_bytes_per_insertion(1, 0, W=0, V=0) - 44 == 32
    assert b.cavity_bytes_per_insertion(0, 1, W=0, V=0) - 44 == 16
    assert b.ball_bytes_per_insertion(26) == 936
    # the per-attempt model: an attempt with no walk and an empty cavity still reads its
    # candidate and point and the two initial vertex records of an empty boundary
    assert b.cavity_bytes_per_attempt(0, 0, 0) == 48 + 32 * 2
    base = b.cavity_bytes_per_attempt(0, 0, 0)
    assert b.cavity_bytes_per_attempt(1, 0, 0) - base == 64
    assert b.cavity_bytes_per_attempt(0, 1, 0) - base == 32 + 16 + 4
    assert b.cavity_bytes_per_attempt(0, 0, 2) - base == 2 * (16 + 16 + 8) + 32
    assert 2900 < b.cavity_bytes_per_attempt(5.7, 20.04, 26.8) < 3100


def test_traffic_is_used_only_for_matching_sources(tmp_path, monkeypatch):
    b = load_bench()
    # a summary carrying the hash of the current kernel sources is read
    summary = ("# summary\n\n- traffic_bytes_per_launch = 414386916\n"
               f"- kernel_source_sha256 = {b.kernel_source_hash()}\n")
    cur = tmp_path / "current.md"
    cur.write_text(summary)
    monkeypatch.setattr(b, "PMC_SUMMARY", str(cur))
    assert b.measured_traffic() == 414386916.0
    # a summary taken on other sources is ignored
    stale = summary.replace("kernel_source_sha256 = ", "kernel_source_sha256 = 0")
    p = tmp_path / "stale.md"
    p.write_text(stale)
    monkeypatch.setattr(b, "PMC_SUMMARY", str(p))
    assert b.measured_traffic() is None
    # as is a missing one
    monkeypatch.setattr(b, "PMC_SUMMARY", str(tmp_path / "missing.md"))
    assert b.measured_traffic() is None


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_cpu_baseline_runs_the_oracle():
    b = load_bench()
    r = b.cpu_baseline(3000, 5)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["unit"] == "tetrahedra/s"
    assert r["value"] > 0 and r["host_threads"] >= 1 and r["cpu"]
    import oracle
    from synth import uniform_points
    rc, tets, _, _ = oracle.delaunay(uniform_points(3000, 5))
    assert rc == 0 and f"{len(tets)} tetrahedra" in r["sample"]


def test_cpu_baseline_over_clouds_stops_at_its_budget():
    b = load_bench()
    import numpy as np
    from synth import batch_clouds
    xyz, off = batch_clouds(6, seed_base=3000, nmin=50, nmax=400)
    off = off.astype(np.int64)
    r = b.cpu_baseline_clouds(xyz, off, [0, 2, 4], budget_s=1e9)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["value"] > 0
    assert r["sample"].startswith("3 of the clouds")
    pts = sum(int(off[c + 1] - off[c]) for c in (0, 2, 4))
    assert f"({pts} points" in r["sample"]
    r = b.cpu_baseline_clouds(xyz, off, [0, 2, 4], budget_s=0.0)
    assert r["sample"].startswith("1 of the clouds")


def test_paper_context_is_quoted_only_where_the_paper_has_the_size():
    b = load_bench()
    assert b.paper_context(10_000_000)["value_at_this_n"] == 31.32e6
    assert b.paper_context(100_000_000)["value_at_this_n"] == 64.40e6
    assert "value_at_this_n" not in b.paper_context(1_000_000)
    assert "context" in b.paper_context(1)["note"]


def _stand_ins(monkeypatch):
    """Replaces the device (torch.cuda, the library's Triangulation and exports) with host
    stand-ins that check the buffers the binding would pass and return fixed statistics."""
    import numpy as np
    import torch

    import paper_1805_08831_amd as pkg
    from paper_1805_08831_amd import dt

    class Stream:
        cuda_stream = 0

    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a, **k: None)
    monkeypatch.setattr(torch.cuda, "current_stream", lambda *a, **k: Stream())
    monkeypatch.setattr(torch.Tensor, "cuda", lambda self, *a, **k: self)
    real_empty = torch.empty
    monkeypatch.setattr(torch, "empty", lambda *a, **k: real_empty(*a, **{x: y for x, y in k.items() if x != "device"}))
    stats = {n: 0 for n, _ in dt.dt_stats._fields_}
    stats.update(attempts=1350, walk_steps=7700, cavity_tets=20000, boundary_facets=26800, inserted=1000,
                 ms_cavity_kernel=12.0, ms_ball_kernel=7.0, cavity_launches=50, ball_launches=50, rounds=50,
                 ms_sort=3.0, ms_insert=20.0, timed_insertions=1000, timed_attempts=1350)

    class Tri:
        def __init__(self, **k):
            self.ctx = 1

        def clear(self):
            pass

        def insert(self, x):
            dt._points(x)

        def insert_batch(self, x, off):
            dt._points(x, int(off[-1]))

        def num_tets(self):
            return 6700

        def stats(self):
            return dict(stats)

        def close(self):
            pass

        def __enter__(self):
            return self

        def __exit__(self, *a):
            pass

    def get_tets(ctx, t=None, nb=None, cap=0):
        dt._out(t, dt._TET_TYPES, 4 * cap, "tets")
        dt._out(nb, dt._NBR_TYPES, 4 * cap, "nbrs")
        return 6700

    monkeypatch.setattr(pkg, "Triangulation", Tri)
    monkeypatch.setattr(pkg, "dt_get_tets", get_tets)
    monkeypatch.setattr(pkg, "dt_get_point_log", lambda ctx: (np.zeros((100, 16), np.float32),
                                                              np.zeros(100, np.float32), np.zeros(100, np.uint8)))
    monkeypatch.setattr(pkg, "dt_train_model", lambda *a, **k: b"model")
    monkeypatch.setattr(pkg, "dt_load_model", lambda ctx, m: None)


CONTRACT_KEYS = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                 "scaling", "vs_baseline", "dtype", "data", "config")


def _run_bench(monkeypatch, capsys, args):
    import json
    b = load_bench()
    monkeypatch.setattr(sys, "argv", ["bench.py"] + args)
    b.main()
    line = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    for k in CONTRACT_KEYS:
        assert k in line, k
    assert line["n_gpus"] == 1 and line["higher_is_better"] is True and line["vs_baseline"] is None
    assert line["data"] == "synthetic" and line["dtype"] == "f64" and "workload" in line["config"]
    return line


def test_bench_line_contract(monkeypatch, capsys):
    """bench.main() on stand-ins for the device (no GPU here): the one JSON line carries every
    field of the output contract, with value = tetrahedra / (ms_per_step / 1000)."""
    _stand_ins(monkeypatch)
    line = _run_bench(monkeypatch, capsys, ["--n", "2000", "--steps", "2", "--warmup", "1", "--no-learned",
                                            "--cpu-sample", "1000", "--u8-steps", "0"])
    assert line["steps"] == 2 and line["warmup"] == 1
    # ms_per_step is printed to 3 decimals: allow that rounding
    assert abs(line["value"] * line["ms_per_step"] / 1000.0 - 6700) <= 6700 * (0.0006 / line["ms_per_step"] + 1e-6)
    r = line["roofline"]
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-4 and "traffic" in r
    assert r["traffic"] is None  # the counters were taken on the 1e7 workload only
    # frac by hand: bytes per insertion x insertions per launch / mean launch time / peak
    C, F = 20000 / 1000, 26800 / 1000
    per = 44 + 4 * 64 + 32 * C + 16 * F + 30 * 32
    assert r["bytes_per_insertion"] == round(per, 1) and r["insertions_per_launch"] == 1000 / 50
    assert abs(r["achieved"] - per * (1000 / 50) / (12.0 / 50 / 1000) / 1e9) < 0.01
    assert "model_per_attempt" in r and line["u8"] is None
    c = line["cpu_baseline"]
    assert c["kind"] == "oracle" and c["cores"] == 1 and c["value"] > 0 and "sample" in c


def test_bench_line_contract_batch_and_mix(monkeypatch, capsys):
    _stand_ins(monkeypatch)
    line = _run_bench(monkeypatch, capsys, ["--workload", "batch", "--clouds", "8", "--chunk", "4",
                                            "--loop-sample", "2", "--steps", "1", "--warmup", "0",
                                            "--no-cpu-baseline"])
    assert line["config"]["calls_per_step"] == 2 and line["config"]["rounds_per_step"] == 100
    assert line["cpu_baseline"] is None
    line = _run_bench(monkeypatch, capsys, ["--workload", "mix", "--mix-scale", "0.001", "--train-samples", "100",
                                            "--steps", "1", "--warmup", "0", "--cpu-mix-scale", "0.05"])
    assert "identical_output" in line["learned"] and line["cpu_baseline"]["kind"] == "oracle"


def test_clock_summary_reads_the_trace_lines():
    """The phase-clock summary adds the rounds' spans and medians and splits large rounds."""
    import bench
    lines = [
        "clocks n=5000 span_us=200.00 walk_us=10.00/20.00/30.00 cav_us=30.00/40.00/90.00 "
        "att_us=40.00/60.00/100.00/150.00 walk_steps=5.00 cav_steps=6.00\n",
        "clocks n=100 span_us=50.00 walk_us=5.00/6.00/7.00 cav_us=15.00/20.00/30.00 "
        "att_us=20.00/25.00/30.00/40.00 walk_steps=3.00 cav_steps=4.00\n",
    ]
    s = bench.summarise_clocks(lines)
    assert s["rounds"] == 2 and s["attempts"] == 5100
    assert s["sum_span_ms"] == 0.25 and s["sum_att_p50_ms"] == 0.06
    assert s["median_attempt_share_of_span"] == round(60 / 250, 4)
    assert s["walk_share_of_median_attempt"] == round(15 / 60, 4)
    assert s["walk_steps_per_attempt"] == round((5 * 5000 + 3 * 100) / 5100, 3)
    assert s["rounds_4096_or_more"]["rounds"] == 1 and s["rounds_below_4096"]["sum_span_ms"] == 0.05
    assert s["rounds_4096_or_more"]["att_us_p50_p90_p99_max_mean"] == [40.0, 60.0, 100.0, 150.0]
    assert bench.summarise_clocks([]) is None
    ball = ("ballclocks n=5000 built=3700 span_us=120.00 test_us=20.00/30.00/50.00 copy_us=5.00/8.00/9.00 "
            "build_us=30.00/40.00/60.00 ball_us=55.00/70.00/90.00/110.00\n")
    s = bench.summarise_clocks(lines + [ball])
    assert s["rounds"] == 2 and s["ball"]["rounds"] == 1 and s["ball"]["sum_span_ms"] == 0.12
    assert s["ball"]["rounds_4096_or_more"]["test_us_p50_p90"] == [20.0, 30.0]
    assert s["ball"]["rounds_4096_or_more"]["ball_us_p50_p90_p99_max"] == [55.0, 70.0, 90.0, 110.0]
