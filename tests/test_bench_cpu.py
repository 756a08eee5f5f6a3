"""The benchmark's CPU-baseline leg on all host cores: CPU-only worker processes run the
unchanged oracle on their own bands of scan rows behind a common start (c1_tiny)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_all_cores_leg_reports_every_worker():
    r = bench.cpu_baseline_all_cores("c1_tiny", 8, 75)
    assert r["kind"] == "oracle" and r["unit"] == "scan-positions/s"
    assert 1 <= r["cores"] <= 16 and r["value"] > 0
    assert f"{r['cores']} concurrent" in r["sample"]


def test_worker_waits_for_the_start_file(tmp_path):
    go = tmp_path / "go"
    p = subprocess.Popen([sys.executable, "-m", "oracle.time_worker", "c1_tiny", "1", "2", str(go)],
                         cwd=ROOT, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)
    try:
        assert p.stdout.readline().strip() == "ready"
        assert p.poll() is None              # still waiting: nothing timed before the start
        go.write_text("")
        out, err = p.communicate(timeout=120)
    finally:
        if p.poll() is None:
            p.kill()
    assert p.returncode == 0, err
    frames, seconds = out.strip().splitlines()[-1].split()
    assert int(frames) == 3 * 2 * 5 and float(seconds) > 0     # 2 raster rows of 5 frames, 3 peaks


def _copy_csrc(tmp_path):
    import shutil
    src = os.path.join(bench.ROOT, "paper_2312_14907_amd", "csrc")
    dst = tmp_path / "paper_2312_14907_amd" / "csrc"
    shutil.copytree(src, dst)
    return dst


def test_counter_hash_follows_the_frame_kernel_code_only(tmp_path):
    """The hash that keys the frame kernel's counter summary covers the code of the frame
    kernel's translation units and the headers they include: a comment edit or an edit
    of another kernel's source leaves it unchanged, a code edit of an included header
    changes it."""
    dst = _copy_csrc(tmp_path)
    files = bench.frame_kernel_sources(str(tmp_path))
    assert "mpbp_frame.hpp" in files and "mpbp_dft.hpp" in files and "mpbp_frames_256.hip" in files
    assert "mpbp_map.hip" not in files and "mpbp_device.hip" not in files
    h0 = bench.kernel_source_hash(str(tmp_path))
    assert h0 == bench.kernel_source_hash()
    with open(dst / "mpbp_dft.hpp", "a") as fh:
        fh.write("\n// a comment\n/* and a block\n comment */\n")
    with open(dst / "mpbp_map.hip", "a") as fh:
        fh.write("\nnamespace mpbp { int unrelated_symbol = 1; }\n")
    assert bench.kernel_source_hash(str(tmp_path)) == h0
    with open(dst / "mpbp_dft.hpp", "a") as fh:
        fh.write("\nnamespace mpbp { constexpr int kChanged = 1; }\n")
    assert bench.kernel_source_hash(str(tmp_path)) != h0
