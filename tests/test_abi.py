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
