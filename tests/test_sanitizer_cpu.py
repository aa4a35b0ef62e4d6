"""The checking build of the library (host code under AddressSanitizer and
UndefinedBehaviorSanitizer, CHEFSI_DEBUG plan-table checks) runs the host-side
ABI driver tests/abi_sanitizer_driver.c without a sanitizer report: argument
validation of every entry point, and the index tables of several plans
(uniform, mixed ALB counts 1..128, length-1 and length-2 periodic dimensions)
checked before any device upload."""
import os
import shutil
import subprocess
import importlib.util

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "llvm", "bin", "clang")


def _build_module():
    spec = importlib.util.spec_from_file_location("_chefsi_build", os.path.join(ROOT, "paper_1606_03416_amd", "build.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


HAVE_HIPCC = shutil.which("hipcc") is not None or os.path.exists("/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not (os.path.exists(CLANG) and HAVE_HIPCC), reason="ROCm toolchain not found")
def test_host_code_under_asan_and_ubsan():
    b = _build_module()
    lib = b.build_sanitized()
    exe = os.path.join(b.SAN_DIR, "abi_driver")
    r = subprocess.run([CLANG, "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-g",
                        "-I" + os.path.join(ROOT, "include"), os.path.join(ROOT, "tests", "abi_sanitizer_driver.c"),
                        "-o", exe, "-L" + b.SAN_DIR, "-lchefsi_san", "-Wl,-rpath," + b.SAN_DIR,
                        "-Wl,-rpath," + os.path.join(b.ROCM, "lib")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out
    assert "0 failures" in out and "AddressSanitizer" not in out and "runtime error" not in out, out
    assert os.path.exists(lib)
