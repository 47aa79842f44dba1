"""Host logic of the benchmark's profile summaries: kernel names as rocprofv3
prints them map to the classes the benchmark times, the timing summary sums
template instances per class, and the counter-based traffic is used only
while the kernel's source is the one the counters were taken from."""
import hashlib
import os

import pytest

import bench


def test_short_names_and_classes():
    a = "void fmmds::k_list_fill<unsigned long, unsigned int, false>(fmmds::ListLevelArgs, int*)"
    b = "fmmds::(anonymous namespace)::k_dense_count(unsigned long const*, unsigned int)"
    assert bench._short_name(a) == "fmmds::k_list_fill<unsigned long, unsigned int, false>"
    assert bench._short_name(b) == "fmmds::k_dense_count"
    assert bench._kernel_class(a) == "list_fill"
    assert bench._kernel_class("void fmmds::k_sort_pass<true, 16>(int)") == "sort_pass"
    assert bench._kernel_class("void fmmds::k_leaf<true, unsigned long>(int)") == "leaf"
    assert bench._kernel_class(b) is None
    assert bench._kernel_class("__amd_rocclr_copyBuffer") is None


def _stats_csv(path):
    rows = [
        ("void fmmds::k_list_fill<unsigned long, unsigned int, false>(int)", 2, 4000000),
        ("void fmmds::k_list_fill<unsigned long, unsigned int, true>(int)", 6, 600000),
        ("fmmds::(anonymous namespace)::k_dense_scan<unsigned long>(int)", 3, 30000),
    ]
    with open(path, "w") as fh:
        fh.write('"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs",'
                 '"StdDev"\n')
        for name, calls, tot in rows:
            fh.write(f'"{name}",{calls},{tot},{tot / calls},10.0,{tot / calls},{tot / calls},0\n')


def test_timing_summary_sums_instances_per_class(tmp_path):
    csv = tmp_path / "run_kernel_stats.csv"
    _stats_csv(csv)
    out = tmp_path / "summary.md"
    bench.kernel_stats_summary(str(csv), str(out), "uniform")
    text = out.read_text()
    # 8 list fill dispatches, 4.6 ms in all: 575 us per dispatch
    assert "| `list_fill` | 8 | 575.0 |" in text
    assert "`fmmds::k_dense_scan<unsigned long>` | 3 | 10.0 |" in text
    assert bench.BUILD_ONLY_FLAGS in text


def test_timing_summary_of_other_runs_has_no_class_table(tmp_path):
    csv = tmp_path / "run_kernel_stats.csv"
    _stats_csv(csv)
    out = tmp_path / "summary.md"
    flags = "--no-cpu-baseline --steps 3 --warmup 1"
    bench.kernel_stats_summary(str(csv), str(out), "uniform", flags)
    text = out.read_text()
    assert "Per kernel class" not in text
    assert f"--workload uniform {flags}" in text
    assert f"--profiled-flags '{flags}'" in text


@pytest.fixture()
def fake_root(tmp_path, monkeypatch):
    src = tmp_path / "kern.hip"
    src.write_text("kernel source v1\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "t.md").write_text(
        "# traffic\n"
        f"traffic list_fill read_bytes_avg=70 write_bytes_avg=1100 dispatches=4 "
        f"source=kern.hip sha={sha}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setitem(bench.TRAFFIC_FILES, "uniform", "t.md")
    return src


def test_counter_traffic_follows_the_source(fake_root):
    got = bench.counter_traffic("uniform", "list_fill")
    assert got == {"read": 70.0, "write": 1100.0, "source": "t.md"}
    assert bench.counter_traffic("uniform", "leaf") is None  # no counters for it
    assert bench.counter_traffic("small", "list_fill") is None  # no summary at all
    fake_root.write_text("kernel source v2\n")  # the kernel changed since
    assert bench.counter_traffic("uniform", "list_fill") is None
