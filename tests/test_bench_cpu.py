"""The benchmark's command line without a GPU: more than one GPU is refused
with a message before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "--gpus 2" in (r.stdout + r.stderr)


def _bench_in(tmp_path, monkeypatch):
    """bench.py's helpers with its repository root moved to tmp_path (a copy
    of the kernel sources, an empty profiles folder), so that nothing
    committed is touched."""
    import importlib.util
    import shutil
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    shutil.copytree(os.path.join(ROOT, "paper_2009_09501_amd", "csrc"), tmp_path / "paper_2009_09501_amd" / "csrc")
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    return b


def test_short_kernel_names(tmp_path, monkeypatch):
    b = _bench_in(tmp_path, monkeypatch)
    assert b._short_kernel("void pstereo::k_warp<true, 2>(pstereo::FrameDesc)") == "k_warp"
    assert b._short_kernel("pstereo::k_rg_merge(pstereo::FrameDesc)") == "k_rg_merge"
    assert b._short_kernel("__amd_rocclr_streamOpsWait") == "__amd_rocclr_streamOpsWait"


def test_percentile_picks_order_statistics(tmp_path, monkeypatch):
    b = _bench_in(tmp_path, monkeypatch)
    xs = list(range(100, 0, -1))  # 100 .. 1, unsorted input
    assert b._pct(xs, 0.5) == 51 and b._pct(xs, 0.99) == 100 and b._pct(xs, 0.0) == 1
    assert b._pct([7.0], 0.99) == 7.0


def test_trace_and_traffic_summaries_round_trip(tmp_path, monkeypatch, capsys):
    """A kernel-stats CSV and two counter CSVs in rocprofv3's column layout
    become per-kernel records under <kernel>@<workload>, tagged with the
    kernel sources' hash, and read back only while the sources are
    unchanged."""
    b = _bench_in(tmp_path, monkeypatch)
    tr = tmp_path / "trace"
    tr.mkdir()
    (tr / "run_kernel_stats.csv").write_text(
        "Name,Calls,TotalDurationNs,AverageNs,Percentage,MinNs,MaxNs\n"
        '"void pstereo::k_warp<true, 2>(pstereo::FrameDesc)",10,250000,25000,50.0,24000,26000\n'
        '"__amd_rocclr_streamOpsWait",20,40000,2000,10.0,500,9000\n')
    b.summarize_trace(str(tr), "4k_test")
    rec = b._profile_record("kernels.json", "k_warp@4k_test")
    assert rec["avg_us"] == 25.0 and rec["calls"] == 10 and rec["min_us"] == 24.0
    assert b._profile_record("kernels.json", "__amd_rocclr_streamOpsWait@4k_test") is None
    rows = "Kernel_Name,Counter_Name,Counter_Value\n"
    fe, wr = tmp_path / "fe", tmp_path / "wr"
    fe.mkdir()
    wr.mkdir()
    (fe / "run_counter_collection.csv").write_text(
        rows + "".join(f'"void pstereo::k_warp<true, 2>(pstereo::FrameDesc)",FETCH_SIZE,{v}\n' for v in (100, 300, 200)))
    (wr / "run_counter_collection.csv").write_text(
        rows + '"void pstereo::k_warp<true, 2>(pstereo::FrameDesc)",WRITE_SIZE,1000\n')
    b.summarize_traffic(str(fe), str(wr), "4k_test", 2.0, 1.0)
    # median FETCH_SIZE 200 KiB x 2 + WRITE_SIZE 1000 KiB x 1
    assert b._traffic("k_warp", "4k_test") == 200 * 1024 * 2 + 1000 * 1024
    # a change to the kernel sources retires the records
    with open(tmp_path / "paper_2009_09501_amd" / "csrc" / "pstereo_api.hip", "a") as fh:
        fh.write("\n// changed\n")
    assert b._traffic("k_warp", "4k_test") is None
    assert b._profile_record("kernels.json", "k_warp@4k_test") is None
    capsys.readouterr()


def test_call_modes_have_paths_and_workloads(tmp_path, monkeypatch):
    b = _bench_in(tmp_path, monkeypatch)
    assert set(b.PATHS) == set(b.WORKLOADS) == {1, 2, 3}
    assert len(set(b.WORKLOADS.values())) == 3
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--stages", "4"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0 and "--stages" in r.stderr
