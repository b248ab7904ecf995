"""The C-ABI library's host code (grid and material assembly, the edge
classification, the source's divergence test, argument validation) built
with AddressSanitizer and UndefinedBehaviorSanitizer on the host side only
(the device code is compiled as usual, and no GPU is touched), then the
no-GPU checks of `tests/test_abi.py` run against that build in a child
process: they must pass with no sanitizer report (any report aborts the
child)."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.timeout(600)
def test_abi_checks_under_host_asan_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    rts = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not os.path.exists(hipcc) or not rts:
        pytest.skip("hipcc or clang's AddressSanitizer runtime not installed")
    csrc = os.path.join(ROOT, "paper_1611_06721_amd", "csrc")
    srcs = sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.cpp")))
    lib = str(tmp_path / "libec_hostsan.so")
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=undefined", "-shared-libsan"]
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-mcode-object-version=5", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           *host_san, "-I", os.path.join(ROOT, "include"), "-I", csrc, "-o", lib, *srcs, "-lrocprofiler-sdk-roctx"]
    subprocess.run(cmd, check=True, capture_output=True)
    child = ("import sys; from paper_1611_06721_amd import _lib; _lib.LIB_PATH = %r; "
             "import pytest; sys.exit(pytest.main(['-q', '-p', 'no:cacheprovider', "
             "'-m', 'not gpu', %r]))" % (lib, os.path.join(ROOT, "tests", "test_abi.py")))
    env = dict(os.environ, LD_PRELOAD=rts[-1], OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", child], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=500)
    report = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, report
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, report
    assert " passed" in r.stdout, report
