"""The host runtime (lbm_runtime.cpp, lbm_batch.cpp, lbm_params.cpp) under
AddressSanitizer (with leak detection) and UndefinedBehaviorSanitizer: the
three sources are compiled with the sanitizers on the host pass only
(-Xarch_host), linked with the library's kernel objects and the harness
tests/host_sanitize.cpp, which drives every entry point that needs no GPU.
CPU only: no device is touched."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2201_04560_amd")
HOST_SOURCES = ["lbm_runtime.cpp", "lbm_batch.cpp", "lbm_params.cpp"]
KERNEL_OBJECTS = ["lbm_step.o", "lbm_aux.o", "lbm_adjoint.o", "lbm_static.o"]


def _hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def test_host_runtime_under_asan_and_ubsan(tmp_path):
    cc = _hipcc()
    if not os.path.exists(cc):
        pytest.skip("hipcc not available")
    from paper_2201_04560_amd import build as b

    objs = [os.path.join(b.OBJ, o) for o in KERNEL_OBJECTS]
    if not all(os.path.exists(o) for o in objs):
        b.build()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    flags = [f"--offload-arch={b.ARCH}", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fPIC"]
    srcs = [os.path.join(PKG, "csrc", s) for s in HOST_SOURCES] + [os.path.join(ROOT, "tests", "host_sanitize.cpp")]
    outs = [str(tmp_path / (os.path.splitext(os.path.basename(s))[0] + ".o")) for s in srcs]

    def compile_one(pair):
        src, out = pair
        return subprocess.run([cc] + flags + san + ["-c", src, "-o", out], capture_output=True, text=True)

    with ThreadPoolExecutor(len(srcs)) as ex:
        for r in ex.map(compile_one, zip(srcs, outs)):
            assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "host_sanitize")
    r = subprocess.run([cc, f"--offload-arch={b.ARCH}"] + san + ["-o", exe] + outs + objs,
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "0 failed expectations" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
