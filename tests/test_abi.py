"""Host-side checks that need no GPU: the C-ABI library loads and exports
every function include/eth.h declares, the Python binding declares each of
them, the host-only calls answer, and the tooling around the kernels
(bench.py's one-GPU contract, the launch geometry the byte-counter reduction
assumes) is consistent.  No kernel is launched."""
import ctypes
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eth.h")
DECL = re.compile(r"^\s*(?:const\s+)?[a-z0-9_]+\s*\*?\s+(eth_[a-z0-9_]+)\s*\(", re.M)


def _declared():
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)   # declarations only, not comments
    names = DECL.findall(text)
    assert len(names) == len(set(names))
    return names


@pytest.fixture(scope="module")
def lib_path():
    from paper_2303_10233_amd import build
    if not os.path.exists(build.LIB):
        build.build(verbose=False)
    return build.LIB


def test_header_declares_the_boundary_calls():
    names = set(_declared())
    for call in ("eth_setup", "eth_destroy", "eth_assemble_rhs", "eth_apply_operator",
                 "eth_apply_preconditioner", "eth_solve", "eth_solve_adjoint", "eth_grad_forcing",
                 "eth_grad_viscosity", "eth_batch_setup", "eth_batch_solve", "eth_batch_destroy",
                 "eth_status_string", "eth_last_error"):
        assert call in names, call


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [name for name in _declared() if not hasattr(lib, name)]
    assert not missing, missing


def test_binding_declares_every_symbol():
    with open(os.path.join(ROOT, "paper_2303_10233_amd", "eth.py")) as f:
        src = f.read()
    undeclared = [name for name in _declared() if f"lib.{name}.argtypes" not in src]
    assert not undeclared, undeclared


def test_binding_fails_loudly_without_the_library(tmp_path):
    """No CPU fallback: loading the product path without a built library is
    an error, not a silent switch to another implementation."""
    from paper_2303_10233_amd import eth
    with pytest.raises(OSError):
        eth.load_library(str(tmp_path / "libeth.so"))


def test_status_strings_without_a_device(lib_path):
    lib = ctypes.CDLL(lib_path)
    lib.eth_status_string.argtypes = [ctypes.c_int]
    lib.eth_status_string.restype = ctypes.c_char_p
    seen = set()
    for code in (0, 1, -1, -2, -3, -4, -5, -6):
        s = lib.eth_status_string(code).decode()
        assert s and s not in seen, (code, s)
        seen.add(s)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = [ln for ln in r.stdout.splitlines() if ln.startswith("{")][-1]
    assert "one GPU" in json.loads(line)["error"]


def test_counter_grid_matches_the_launch_geometry():
    """traffic.mq_grid must name the work-items of the fused step's launch:
    ceil(n / tile)^2 blocks (the last tiles own node n) of 64 * ceil(QW^2 / 64)
    threads for tiles below 32 (QW = tile / 2 + 10 * steps) and 1024 threads
    for larger tiles."""
    from paper_2303_10233_amd.traffic import mq_grid
    assert mq_grid(256, 16) == 16 * 16 * 384
    assert mq_grid(256, 16, 2) == 16 * 16 * 832
    assert mq_grid(256, 32) == 8 * 8 * 1024
    assert mq_grid(250, 16) == 16 * 16 * 384
    assert mq_grid(257, 64) == 5 * 5 * 1024
    assert mq_grid(256, 24) == 11 * 11 * 512
    assert mq_grid(256, 24, 2) == 11 * 11 * 1024
    from paper_2303_10233_amd.traffic import apply_grid
    assert apply_grid(2048) == 65 * 257 * 256   # 64 x 16 node tiles of 4097^2 nodes, 256 threads


def _counter_csv(path, counter, rows):
    with open(path, "w") as f:
        f.write("Kernel_Name,Grid_Size,Counter_Name,Counter_Value\n")
        for name, grid, kib in rows:
            f.write(f'"{name}",{grid},{counter},{kib}\n')


def test_traffic_reduction_scales_by_the_copy_calibration(tmp_path):
    """The byte-counter reduction: each counter of the target kernel is
    averaged over its dispatches and scaled by bytes / counter of the large
    copy (FETCH_SIZE reading half the copied bytes gives the factor 2), and
    the record names the sha256 of the kernel's source file."""
    import hashlib
    from paper_2303_10233_amd.traffic import copy_grid, mq_grid
    half = 335708184.0                                   # bytes read = bytes written by the copy
    name = "void eth::k_mq_cheb_fused<float, 16, 1>(eth::Geo, float*)"
    g = mq_grid(256, 16)
    fetch_rows = [("k_copy(long long)", copy_grid(2048), half / 1024 / 2),
                  ("k_copy(long long)", copy_grid(256), 1000.0),
                  (name, g, 2000.0), (name, g, 3000.0),     # mean 2500 KiB
                  (name, g + 64, 9999.0)]                   # another grid: ignored
    write_rows = [("k_copy(long long)", copy_grid(2048), half / 1024),
                  ("k_copy(long long)", copy_grid(256), 2000.0),
                  (name, g, 1500.0), (name, g, 1500.0)]
    _counter_csv(tmp_path / "f.csv", "FETCH_SIZE", fetch_rows)
    _counter_csv(tmp_path / "w.csv", "WRITE_SIZE", write_rows)
    rec = {"n": 256, "launches": [
        {"kernel": "k_mq_cheb_fused", "n": 256, "bytes_per_launch": 2631700.0, "mq_tile": 16},
        {"kernel": "k_copy", "n": 2048, "bytes_per_launch": 2 * half},
        {"kernel": "k_copy", "n": 256, "bytes_per_launch": 10526768.0}]}
    (tmp_path / "l.json").write_text("log line\n" + json.dumps(rec) + "\n")
    out = tmp_path / "t.json"
    r = subprocess.run([sys.executable, "-m", "paper_2303_10233_amd.traffic", "--fetch", str(tmp_path / "f.csv"),
                        "--write", str(tmp_path / "w.csv"), "--launches", str(tmp_path / "l.json"),
                        "--out", str(out)], capture_output=True, text=True, timeout=60, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    d = json.loads(out.read_text())
    assert d["dispatches"] == {"fetch": 2, "write": 2}
    assert d["copy_calibration"]["fetch_scale"] == pytest.approx(2.0)
    assert d["copy_calibration"]["write_scale"] == pytest.approx(1.0)
    assert d["bytes_per_launch"] == pytest.approx(2500.0 * 1024 * 2 + 1500.0 * 1024, abs=0.1)
    with open(os.path.join(ROOT, "paper_2303_10233_amd", "csrc", "k_mq.hip"), "rb") as f:
        assert d["source_sha256"] == hashlib.sha256(f.read()).hexdigest()


def test_bench_reports_counted_traffic_only_for_the_counted_kernel():
    """bench.py's roofline.traffic comes from the committed counter record
    only while it describes the timed kernel: same template variant and the
    same source file (sha256); otherwise null."""
    sys.path.insert(0, ROOT)
    import bench
    with open(os.path.join(ROOT, "profiles", "k_mq_cheb_fused_stokes256_traffic.json")) as f:
        rec = json.load(f)
    import hashlib
    with open(os.path.join(ROOT, "paper_2303_10233_amd", "csrc", rec["source"]), "rb") as f:
        current = hashlib.sha256(f.read()).hexdigest() == rec["source_sha256"]
    v = bench.measured_traffic("k_mq_cheb_fused", 256, rec["kernel"])
    if current:
        assert v == rec["bytes_per_launch"] and v > rec["algorithmic_bytes_per_launch"]
    else:   # the kernel changed after the counters were read
        assert v is None
    assert bench.measured_traffic("k_mq_cheb_fused", 256, "k_mq_cheb_fused<float, 32, 1>") is None
    assert bench.measured_traffic("k_mq_cheb_fused", 512, rec["kernel"]) is None
    assert bench.measured_traffic("k_dot", 256, None) is None
