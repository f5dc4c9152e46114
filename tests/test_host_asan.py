"""The host side of the runtime under AddressSanitizer and UBSan (no GPU
needed): eth_runtime.hip, eth_noalloc.hip, eth_step.hip and eth_step_asm.hip
are rebuilt with the sanitizers on their host code only (-Xarch_host), linked
with the other objects, and a child Python process with the ASan runtime
preloaded drives every call that answers without a device (status strings,
argument checks, failing set-ups with their clean-up, and the step's host
assembly of every matrix kind, on meshes large enough for its multi-threaded
row fill).  Opt-in (ETH_ASAN=1): the instrumented build takes about a
minute."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
@pytest.mark.skipif(os.environ.get("ETH_ASAN") != "1", reason="set ETH_ASAN=1 (instrumented build, ~1 min)")
def test_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2303_10233_amd import build
    build.build(verbose=False)
    hipcc = build.HIPCC
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
    objs = []
    for src in build.SOURCES:
        obj = os.path.join(build.BUILD, os.path.splitext(src)[0] + ".o")
        if src in ("eth_runtime.hip", "eth_noalloc.hip", "eth_step.hip", "eth_step_asm.hip"):
            obj = str(tmp_path / (os.path.splitext(src)[0] + ".asan.o"))
            cmd = [hipcc, *build.FLAGS, *san, "-c", os.path.join(build.CSRC, src), "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-2000:]
        objs.append(obj)
    lib = str(tmp_path / "libeth_asan.so")
    r = subprocess.run([hipcc, f"--offload-arch={build.ARCH}", "-shared", "-fPIC", "-fsanitize=address,undefined",
                        *objs, "-o", lib, "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
                        "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    rt = subprocess.run([hipcc, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    assert os.path.exists(rt), rt
    driver = r"""
import ctypes, sys
sys.path.insert(0, %r)
from paper_2303_10233_amd import eth
L = eth.load_library(%r)
for code in (0, 1, 2, -1, -2, -3, -4, -5, -6, 99):
    assert L.eth_status_string(code)
d = eth.ProblemDesc()
h = ctypes.c_void_p()
for n in (1, 0, -3):                      # invalid sizes: refused before any device call
    d.n = n
    assert L.eth_setup(ctypes.byref(d), ctypes.byref(h)) == eth.EINVAL and not h.value
    assert L.eth_last_error(None)
d.n = 8; d.x0, d.x1, d.y0, d.y1 = 0.0, 1.0, 0.0, 2.0
assert L.eth_setup(ctypes.byref(d), ctypes.byref(h)) == eth.EINVAL       # not square
d.y1 = 1.0; d.nu = -1.0
assert L.eth_setup(ctypes.byref(d), ctypes.byref(h)) == eth.EINVAL
d.nu = 1.0; d.mq_tile = 7
assert L.eth_setup(ctypes.byref(d), ctypes.byref(h)) == eth.EINVAL
d.mq_tile = 0
rc = L.eth_setup(ctypes.byref(d), ctypes.byref(h))   # no GPU here: fails in the runtime, cleans up
assert rc < 0 and not h.value, rc
assert L.eth_destroy(None) == eth.EINVAL
assert L.eth_misfit_noalloc(None, None, None, None, None, 1, 1) == eth.EINVAL
import numpy as np
for m, ch in ((4, False), (32, False), (6, True)):
    nv = eth.step_host_layout(m, channel=ch)["q2_ij"].shape[0]
    w = np.linspace(-1.0, 1.0, 2 * nv)
    for k in (eth.STEP_K, eth.STEP_F1, eth.STEP_MQ, eth.STEP_Q1, eth.STEP_AP, eth.STEP_P, eth.STEP_PQ, eth.STEP_RHS):
        eth.step_host_matrix(m, k, channel=ch, nu=0.02, wind=w)
print("ASAN_DRIVER_OK")
""" % (ROOT, lib)
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([sys.executable, "-c", driver], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "ASAN_DRIVER_OK" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
