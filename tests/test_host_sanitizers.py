"""The host half of the C ABI (setup, geometry and stretch tables,
nested-dissection plans, buffer queries, validation and the state machine)
built with g++ under AddressSanitizer and UndefinedBehaviorSanitizer (leak
checks on) and driven by tests/host/abi_sanitize_check.cpp.  CPU only: the
harness calls nothing that launches a kernel."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1508_02897_amd", "csrc")
HIPLIB = "/opt/rocm/lib/libamdhip64.so"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(HIPLIB),
                    reason="needs g++ and the HIP runtime library")
def test_host_abi_clean_under_asan_and_ubsan(tmp_path):
    flags = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
             "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]
    srcs = [os.path.join(CSRC, "hddm_host.cpp"), os.path.join(CSRC, "hddm_nd_plan.cpp"),
            os.path.join(ROOT, "tests", "host", "abi_sanitize_check.cpp")]
    objs = []
    for src in srcs:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run(["g++"] + flags + ["-c", src, "-o", obj], check=True, timeout=600)
        objs.append(obj)
    exe = str(tmp_path / "check")
    subprocess.run(["g++", "-fsanitize=address,undefined"] + objs +
                   ["-o", exe, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib",
                    "-Wl,--unresolved-symbols=ignore-in-object-files"], check=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout, r.stderr)
    assert r.returncode == 0
    assert "0 failures" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
