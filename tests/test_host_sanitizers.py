"""The host code of the C ABI under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only: the device code is built as
usual).  qoc_api.cpp is compiled with the sanitizers, linked with the
library's other objects and a driver (tests/host/abi_driver.cpp) that runs
every validation path of qoc_create, the (p, n) rule and the argument
checks of the other entry points; no GPU is needed (a valid problem stops
at the device check).  Leak detection is off: the HIP runtime's own
initialisation allocations are not this code's."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1612_04929_amd", "csrc")
OUT = os.path.join(ROOT, "paper_1612_04929_amd", "_build_san")


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


def clangxx():
    c = "/opt/rocm/llvm/bin/clang++"
    return c if os.path.exists(c) else None


@pytest.fixture(scope="module")
def driver():
    if not hipcc() or not clangxx():
        pytest.skip("hipcc / clang++ of ROCm not found")
    from paper_1612_04929_amd import build as qbuild
    objs_dir = qbuild.BUILD_DIR
    others = [os.path.join(objs_dir, s + ".o") for s in qbuild.SOURCES if s != "qoc_api.cpp"]
    if not all(os.path.exists(o) for o in others):
        qbuild.build()
    os.makedirs(OUT, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
    api_o = os.path.join(OUT, "qoc_api_san.o")
    drv_o = os.path.join(OUT, "abi_driver_san.o")
    exe = os.path.join(OUT, "abi_driver")
    cmd = [hipcc(), "-x", "hip"] + qbuild.FLAGS + ["-g", "-O1"] + san + \
        ["-c", os.path.join(CSRC, "qoc_api.cpp"), "-o", api_o]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    san_host = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                "-fno-sanitize-recover=all"]
    r = subprocess.run([clangxx(), "-std=c++17", "-g", "-O1"] + san_host +
                       ["-c", os.path.join(HERE, "host", "abi_driver.cpp"), "-o", drv_o],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([clangxx()] + san_host + [drv_o, api_o] + others +
                       ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


def test_abi_host_code_under_asan_and_ubsan(driver):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "abi driver: ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out
