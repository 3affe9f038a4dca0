"""Host-side checks of the measurement harness: the rocprofv3 summaries that bench.py reads
(traffic per dispatch, only for the kernel source they were taken on), the kernel-stats
aggregation, and the single-GPU guard of bench.py. No GPU needed."""
import os
import subprocess
import sys

from paper_1808_01364_amd import prof_summary as ps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _traffic_file(tmp_path, sha):
    p = tmp_path / "traffic.txt"
    p.write_text("\n".join([
        "# HBM traffic per dispatch",
        "command: test",
        f"kernels_hip_sha256: {sha}",
        "copy_kernel: k_copy",
        "",
        "kernel                 dispatches   fetch_KiB   write_KiB  traffic_bytes",
        "k_skeletonize                   2        10.0        20.0        1000",
        "k_skeletonize_x                 1        10.0        20.0        9999",
        "k_apply_trsv_up                 3         1.0         1.0         300",
        "k_apply_gemv_up                 1         1.0         1.0         700",
    ]) + "\n")
    return str(p)


def test_read_traffic_weights_by_dispatches(tmp_path):
    path = _traffic_file(tmp_path, ps.kernel_source_sha())
    assert ps.read_traffic(path, "k_skeletonize") == 1000.0
    # several kernels of one class: dispatch-weighted mean, (3 * 300 + 1 * 700) / 4
    assert ps.read_traffic(path, ("k_apply_trsv_up", "k_apply_gemv_up")) == 400.0


def test_read_traffic_refuses_stale_or_missing(tmp_path):
    assert ps.read_traffic(_traffic_file(tmp_path, "0" * 64), "k_skeletonize") is None
    path = _traffic_file(tmp_path, ps.kernel_source_sha())
    assert ps.read_traffic(path, "k_not_listed") is None
    assert ps.read_traffic(str(tmp_path / "missing.txt"), "k_skeletonize") is None


def test_short_names_merge_template_forms():
    assert ps._short("void rhif::k_skeletonize<4, double, 16>(rhif::SkelDesc const*, int)") == "k_skeletonize"
    assert ps._short("rhif::k_chol_lead(rhif::FrontDesc const*, double*)") == "k_chol_lead"
    assert ps._short("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_stats_aggregates_forms_of_one_kernel(tmp_path):
    csv_path = tmp_path / "stats.csv"
    csv_path.write_text("\n".join([
        '"Name","Calls","TotalDurationNs","AverageNs","Percentage","MinNs","MaxNs","StdDev"',
        '"void rhif::k_skeletonize<4, double, 16>(int)",2,4000,2000,40.0,1000,3000,0',
        '"void rhif::k_skeletonize<3, double, 96>(int)",1,5000,5000,50.0,5000,5000,0',
        '"rhif::k_copy(long, double const*, double*)",4,1000,250,10.0,200,300,0',
    ]) + "\n")
    out = tmp_path / "summary.txt"
    ps.stats(str(csv_path), str(out), "cmd")
    rows = {ln.split()[0]: ln.split() for ln in out.read_text().splitlines()[5:]}
    sk = rows["k_skeletonize"]
    assert int(sk[1]) == 3 and float(sk[2]) == 9.0        # calls, total_us
    assert float(sk[3]) == 3.0                             # avg_us over both forms
    assert float(sk[4]) == 1.0 and float(sk[5]) == 5.0     # min_us, max_us
    assert list(rows)[0] == "k_skeletonize"                # sorted by total time


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
