"""Address and undefined-behaviour sanitizer runs of the CPU code:

* the oracle, built with -fsanitize=address,undefined and driven through
  every entry point (tests/sanitize/oracle_driver.c);
* the host code of the HIP library's C ABI (argument validation, interaction
  lists, the autotune cache file, option handling), built for the host with
  the same sanitizers and exercised without a device by
  tests/sanitize/host_driver.cpp.

Both builds go to a temporary directory; a sanitizer report fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=timeout)
    return r.returncode, r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc unavailable")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    rc, out = _run(["gcc", "-std=c99", *SAN, "-o", exe, os.path.join(ROOT, "oracle", "fmm_oracle.c"),
                    os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-lm"])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    rc, out = _run([exe], env=env)
    assert rc == 0 and "every entry point ran" in out, out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out


HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc unavailable")
def test_host_abi_under_asan_ubsan(tmp_path):
    """fmm_api.cpp compiled for the host only, with the sanitizers on the host
    side of every hipcc line, driven through the argument checks."""
    host_san = []
    for f in ("address", "undefined"):
        host_san += ["-Xarch_host", f"-fsanitize={f}"]
    common = ["-x", "hip", "--offload-host-only", "-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer",
              "-I" + os.path.join(ROOT, "include"), *host_san]
    objs = []
    for src in (os.path.join(ROOT, "paper_2606_13793_amd", "csrc", "fmm_api.cpp"),
                os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp")):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        rc, out = _run([HIPCC, *common, "-c", src, "-o", obj])
        assert rc == 0, out
        objs.append(obj)
    exe = str(tmp_path / "host_driver")
    rc, out = _run([HIPCC, *host_san, "-o", exe, *objs, "-L/opt/rocm/lib", "-lamdhip64"])
    assert rc == 0, out
    # the HIP runtime keeps allocations until exit; leaks are not what this checks
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1",
               HIP_VISIBLE_DEVICES="")
    rc, out = _run([exe], env=env)
    assert rc == 0 and "every call returned the expected status" in out, out
    assert "runtime error" not in out and "AddressSanitizer" not in out, out
