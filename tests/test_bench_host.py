"""The measurement script's host logic, without a GPU: the one-GPU refusal,
the algorithmic bytes per kernel against the plan's totals, and the
summaries written from rocprofv3 CSV output (calibration by the copy
kernel, per-launch traffic, stale-source detection)."""
import csv
import json
import os
import subprocess
import sys

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


@pytest.mark.parametrize("name", ["c1", "c2", "c3"])
def test_kernel_bytes_add_up_to_the_plan_totals(name):
    """Per-kernel algorithmic bytes (input maximum aside, which reads the
    input once more) sum to the plan's bytes per direction."""
    from paper_1604_07651_amd import hrt
    desc = synth.config_desc(name)
    info = hrt.describe(desc)
    b = bench.kernel_alg_bytes(info, desc)
    assert len(b) == len(bench.STAGE_KERNELS) == 12
    assert abs(sum(b[1:6]) - info["alg_bytes_fwd"]) <= 1e-9 * info["alg_bytes_fwd"]
    assert abs(sum(b[7:12]) - info["alg_bytes_adj"]) <= 1e-9 * info["alg_bytes_adj"]


def _write_csv(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_profile_summaries_from_csv(tmp_path, monkeypatch):
    """A plain 256 MiB copy whose FETCH_SIZE reads half its bytes sets the
    read factor to 2 (the largest copy dispatch counts, small copies do
    not); a kernel's bytes per launch are its per-dispatch average times the
    factors; the stored traffic is used only for the same kernel sources."""
    h = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "profiles" / "c3_traffic.json"))
    spread = "void hrt::k_spread<1, false>(hrt::DevGeo, hrt::DevGeo const*, int2 const*, float const*)"
    copy = "__amd_rocclr_copyBuffer"
    _write_csv(str(tmp_path / "trace" / "run_kernel_stats.csv"),
               ["Name", "Calls", "AverageNs", "Percentage"],
               [[spread, 40, 30000.0, 60.0], [copy, 3, 1000.0, 1.0]])
    fetch_kib = 256 * 1024 // 2
    _write_csv(str(tmp_path / "fetch" / "run_counter_collection.csv"),
               ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"],
               [[copy, 1, "FETCH_SIZE", 8.0], [copy, 2, "FETCH_SIZE", fetch_kib],
                [spread, 3, "FETCH_SIZE", 1000.0], [spread, 4, "FETCH_SIZE", 3000.0]])
    _write_csv(str(tmp_path / "write" / "run_counter_collection.csv"),
               ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"],
               [[copy, 1, "WRITE_SIZE", 4.0], [copy, 2, "WRITE_SIZE", 256 * 1024],
                [spread, 3, "WRITE_SIZE", 500.0], [spread, 4, "WRITE_SIZE", 500.0]])
    bench.summarize_profiles(str(tmp_path / "trace"), str(tmp_path / "fetch"),
                             str(tmp_path / "write"), ["cmd"], h)
    t = json.load(open(bench.TRAFFIC_FILE))
    assert t["fetch_factor"] == pytest.approx(2.0)
    assert t["write_factor"] == pytest.approx(1.0)
    k = t["kernels"]["k_spread<1, false>"]
    assert k["hbm_bytes"] == pytest.approx(2000.0 * 1024 * 2 + 500.0 * 1024)
    assert bench.stored_traffic("k_spread<1, false>") == pytest.approx(k["hbm_bytes"])
    md = open(tmp_path / "profiles" / "c3_kernels.md").read()
    assert "| k_spread<1, false> | 40 | 30.00 |" in md
    # counters taken on other sources are not used
    t["source_hash"] = "0" * 16
    json.dump(t, open(bench.TRAFFIC_FILE, "w"))
    assert bench.stored_traffic("k_spread<1, false>") is None


def test_kernel_hash_ignores_comments_only(tmp_path, monkeypatch):
    """The stored counters follow the kernels' code: a comment or blank-line
    edit keeps kernel_source_hash, a change of code (string literals
    included) changes it."""
    src = tmp_path / "paper_1604_07651_amd" / "csrc"
    src.mkdir(parents=True)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (src / "k.hip").write_text('int a = 1;  // one\nconst char* s = "x // y";\n')
    h0 = bench.kernel_source_hash()
    (src / "k.hip").write_text('/* block\n comment */\nint a = 1;\n\n'
                               'const char* s = "x // y";  // trailing\n')
    assert bench.kernel_source_hash() == h0
    (src / "k.hip").write_text('int a = 2;\nconst char* s = "x // y";\n')
    assert bench.kernel_source_hash() != h0
    (src / "k.hip").write_text('int a = 1;\nconst char* s = "x // z";\n')
    assert bench.kernel_source_hash() != h0


def test_batch_trace_summary(tmp_path, monkeypatch):
    """The batch trace summary keeps the batched kernels only and gives each
    its time per forward+adjoint pass (launches x average over the passes
    the trace holds: the timed ones and the warm-up)."""
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    (tmp_path / "profiles").mkdir()
    _write_csv(str(tmp_path / "trace" / "run_kernel_stats.csv"),
               ["Name", "Calls", "AverageNs", "Percentage"],
               [["void hrt::k_spread<1, true>(hrt::DevGeo, int2 const*, float const*)", 11,
                 500000.0, 40.0],
                ["void hrt::k_spread<1, false>(hrt::DevGeo, int2 const*, float const*)", 3,
                 30000.0, 1.0],
                ["__amd_rocclr_copyBuffer", 4, 3000.0, 0.1]])
    bench.summarize_batch_trace(str(tmp_path / "trace"), ["cmd"], "abc", 10)
    text = (tmp_path / "profiles" / "c4_batch_kernels.md").read_text()
    assert "| k_spread<1, true> | 11 | 500.00 | 500.0 | 100.0 % |" in text
    assert "k_spread<1, false>" not in text and "copyBuffer" not in text
    assert "0.500 ms" in text and "Kernel source hash: abc" in text
