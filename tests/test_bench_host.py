"""Host logic of bench.py: the byte model of the roofline figure, the
counter summary (FETCH_SIZE / WRITE_SIZE scaled by a copy of known size,
the largest launch grid of each kernel) and the lookup of the timed
kernel's line in it, and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_apply_bytes_per_node():
    # 5 blocks x 21 floats + 7 node records read, 6 written (24 B) + the
    # 16-float regulariser record; batched: u neither read nor written
    assert bench.apply_bytes(0, 1, 2) == 420 + 13 * 24 + 64 == 796
    assert bench.apply_bytes(0, 1, 2, batched=True) == 796 - 48
    # matrix-free: the 21 distinct block floats per pixel on top
    assert bench.apply_bytes(10, 1, 0) == 10 * 84 + 376
    G0, N0 = 160 * 120, 640 * 480
    assert bench.apply_bytes(N0, G0, 2) == 15283200


def test_kernel_prefix():
    assert bench.pcg_kernel_prefix(False, 2, 4, 2) == "k_pcg<false, false, 0, 2"
    assert bench.pcg_kernel_prefix(True, 0, 4, 1) == "k_pcg<true, false, 4, 1"


def _summary(sha):
    return [
        "# header",
        f"source_sha256 = {sha}",
        "# k_pcg<false, false, 0, 2, true>, launch grid 76800 threads: ...",
        "traffic_bytes_per_launch[k_pcg<false, false, 0, 2, true>] = 111",
        "# k_pcg<false, false, 0, 2, false>, launch grid 19200 threads: ...",
        "traffic_bytes_per_launch[k_pcg<false, false, 0, 2, false>] = 222",
        "# k_pcg<false, false, 0, 3, false>, launch grid 5120 threads: ...",
        "traffic_bytes_per_launch[k_pcg<false, false, 0, 3, false>] = 333",
    ]


def test_traffic_lookup_picks_the_level0_launch():
    lines = _summary("abc")
    # both WD instances of V = 2: the one of the largest grid (level 0)
    assert bench.traffic_lookup(lines, "k_pcg<false, false, 0, 2", "abc") == (
        "k_pcg<false, false, 0, 2, true>", 111)
    assert bench.traffic_lookup(lines, "k_pcg<false, false, 0, 3", "abc") == (
        "k_pcg<false, false, 0, 3, false>", 333)
    # no such kernel; a summary of another kernel source
    assert bench.traffic_lookup(lines, "k_pcg<false, false, 0, 1", "abc") == (None, None)
    assert bench.traffic_lookup(lines, "k_pcg<false, false, 0, 2", "xyz") == (None, None)
    # a prefix must end at a template argument: V = 2 is not V = 20
    lines += ["# k_pcg<false, false, 0, 20, true>, launch grid 99999 threads: ...",
              "traffic_bytes_per_launch[k_pcg<false, false, 0, 20, true>] = 444"]
    assert bench.traffic_lookup(lines, "k_pcg<false, false, 0, 2", "abc")[1] == 111


def _csv(path, counter, rows):
    with open(path, "w") as f:
        f.write("Kernel_Name,Grid_Size,Counter_Name,Counter_Value\n")
        for name, grid, value in rows:
            f.write(f'"{name}",{grid},{counter},{value}\n')


def test_traffic_report_scales_by_the_copy_probe(tmp_path, capsys):
    name = "void (anonymous namespace)::k_pcg<true, false, 0, 0, true>(FrameMap, TileCfg, int, int, int)"
    # the copy of 1 MiB reads 512 KiB by FETCH_SIZE and 1024 KiB by WRITE_SIZE
    # a grid only the fetch run saw (the runs autotune separately) is
    # skipped, and so is the first-iteration kernel (FIRST = true)
    first = "void (anonymous namespace)::k_pcg<true, true, 0, 0, true, false>(FrameMap, TileCfg, int, int, int)"
    fetch = [("__amd_rocclr_copyBuffer", 256, 512.0),
             (name, 1000, 100.0), (name, 1000, 102.0), (name, 500, 7.0), (name, 4000, 9.0),
             (first, 1000, 5.0)]
    write = [("__amd_rocclr_copyBuffer", 256, 1024.0),
             (name, 1000, 50.0), (name, 1000, 52.0), (name, 500, 3.0), (first, 1000, 5.0)]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _csv(fp, "FETCH_SIZE", fetch)
    _csv(wp, "WRITE_SIZE", write)
    bench.traffic_report(str(fp), str(wp), [], 1)
    out = capsys.readouterr().out.splitlines()
    line = [l for l in out if l.startswith("traffic_bytes_per_launch[")]
    assert line == ["traffic_bytes_per_launch[k_pcg<true, false, 0, 0, true>] = "
                    f"{int(round((101.0 * 2.0 + 51.0 * 1.0) * 1024))}"]
    assert any("launch grid 1000 threads" in l for l in out)
    got = bench.traffic_lookup(out, "k_pcg<true, false, 0, 0", bench.source_hash())
    assert got[1] == int(round((101.0 * 2.0 + 51.0) * 1024))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
