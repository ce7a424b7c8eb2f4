"""The serving engine's scheduler under host sanitizers (no GPU).

csrc/dop_serve.cpp (scheduler thread, condition variables, first-fit arena,
ticket table) is compiled as host code together with host stand-ins for the HIP
runtime and the GPU enqueue (tests/c/serve_host_stubs.cpp), and the
multi-threaded stress driver tests/c/serve_stress.cpp runs it through the C
ABI with the mock executor: once under ThreadSanitizer, once under
AddressSanitizer + UndefinedBehaviorSanitizer.  Any sanitizer report fails.
Skipped when the compiler or a sanitizer runtime is missing.

The compiler is the LLVM clang++ that ships with ROCm (its ThreadSanitizer
intercepts pthread_cond_clockwait, which std::condition_variable::wait_for
uses with glibc 2.30 and later; GCC 11's does not, and then reports the
waiting thread as still holding the mutex), else g++.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = [os.path.join(ROOT, "paper_2505_22313_amd", "csrc", "dop_serve.cpp"),
           os.path.join(ROOT, "tests", "c", "serve_host_stubs.cpp"),
           os.path.join(ROOT, "tests", "c", "serve_stress.cpp")]
ROCM_INCLUDE = "/opt/rocm/include"
ROCM_CLANG = "/opt/rocm/llvm/bin/clang++"


def _compiler():
    if os.path.exists(ROCM_CLANG):
        return ROCM_CLANG
    return shutil.which("g++")

CONFIGS = {
    "thread": (["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1 exitcode=66"}),
    "address_undefined": (["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
                          {"ASAN_OPTIONS": "detect_leaks=1 halt_on_error=1",
                           "UBSAN_OPTIONS": "print_stacktrace=1 halt_on_error=1"}),
}
REPORT_MARKERS = ("WARNING: ThreadSanitizer", "ERROR: AddressSanitizer", "ERROR: LeakSanitizer",
                  "runtime error:")


def _sanitizer_works(flags, tmp_path):
    src = tmp_path / "probe.cpp"
    src.write_text("#include <thread>\nint main(){int x=0;std::thread t([&]{x=1;});t.join();"
                   "return x-1;}\n")
    exe = tmp_path / "probe"
    r = subprocess.run([_compiler(), "-pthread", *flags, str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    if r.returncode != 0:
        return False
    return subprocess.run([str(exe)], capture_output=True).returncode == 0


@pytest.mark.parametrize("name", sorted(CONFIGS))
def test_serve_scheduler_under_sanitizer(name, tmp_path):
    if _compiler() is None or not os.path.isdir(ROCM_INCLUDE):
        pytest.skip("no host C++ compiler or no HIP headers")
    flags, env_extra = CONFIGS[name]
    if not _sanitizer_works(flags, tmp_path):
        pytest.skip(f"the {name} sanitizer runtime is not usable here")
    exe = tmp_path / f"serve_stress_{name}"
    cmd = [_compiler(), "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread", *flags,
           "-D__HIP_PLATFORM_AMD__", "-I", ROCM_INCLUDE, *SOURCES, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, **env_extra)
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-6000:]
    assert not any(m in out for m in REPORT_MARKERS), out[-6000:]
    assert "serve stress: ok" in r.stdout
