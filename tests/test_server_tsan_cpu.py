"""The job server's threads under ThreadSanitizer, on the CPU.

api.cpp and serve.cpp are compiled for the host against a stand-in HIP
runtime (`tests/host_fake/hip/hip_runtime.h`: device memory is host memory,
streams and events complete at once) with the device launchers replaced by
`tests/host_fake/fake_kernels.cpp` (no kernel runs; steps advance the host
clock as the real launchers do).  `server_race_driver.cpp` then runs the
server's builder and stepper threads against four client threads that
submit, query, cancel, wait for, read and release jobs while a collector
drains dpsnn_server_wait_any, with and without allocator callbacks, and
checks that every job is accounted for and every byte returned.  Any
ThreadSanitizer report fails the test.  Needs a clang with the TSan runtime
(the ROCm LLVM ships one); gcc 11's runtime does not intercept the
condition-variable waits of its own libstdc++ and reports false races."""
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = os.path.join(ROOT, "tests", "host_fake")


def _clang():
    for c in ("/opt/rocm/llvm/bin/clang++", "clang++"):
        r = subprocess.run([c, "--version"], capture_output=True)
        if r.returncode == 0:
            return c
    return None


def test_server_threads_under_tsan(tmp_path):
    cxx = _clang()
    if cxx is None:
        pytest.skip("clang++ not available")
    probe = tmp_path / "p.cpp"
    probe.write_text("#include <thread>\nint main() { std::thread t([] {}); t.join(); }\n")
    if subprocess.run([cxx, "-fsanitize=thread", "-pthread", str(probe), "-o", str(tmp_path / "p")],
                      capture_output=True).returncode != 0:
        pytest.skip("no ThreadSanitizer runtime for clang++")
    flags = ["-std=c++17", "-O1", "-g", "-fsanitize=thread", "-Wno-unknown-pragmas",
             "-Wno-division-by-zero", "-I", FAKE, "-I", os.path.join(ROOT, "include"),
             "-I", os.path.join(ROOT, "paper_1310_8478_amd", "csrc")]
    srcs = [os.path.join(ROOT, "paper_1310_8478_amd", "csrc", "api.cpp"),
            os.path.join(ROOT, "paper_1310_8478_amd", "csrc", "serve.cpp"),
            os.path.join(FAKE, "fake_kernels.cpp"), os.path.join(FAKE, "server_race_driver.cpp")]
    objs = []
    for s in srcs:
        o = str(tmp_path / (os.path.basename(s) + ".o"))
        subprocess.check_call([cxx, *flags, "-c", s, "-o", o])
        objs.append(o)
    exe = str(tmp_path / "race")
    subprocess.check_call([cxx, "-fsanitize=thread", "-pthread", *objs, "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, TSAN_OPTIONS="halt_on_error=0 exitcode=66"))
    assert "ThreadSanitizer" not in r.stderr, r.stderr[:6000]
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr[:3000]
