"""The event sort of the ORDERED fold (sift_events / sort_events in step.hip)
compiled for the host from the kernel source itself and checked against
std::sort: random distinct keys of 0 .. 2000 events, weights moving with their
keys, nothing written outside the range; built with AddressSanitizer and
UndefinedBehaviorSanitizer where gcc has them."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r"""
#include <algorithm>
#include <cstdio>
#include <random>
#include <set>
#include <vector>
int main() {
    std::mt19937_64 g(7);
    const unsigned long long guard = 0xAAAAAAAAAAAAAAAAull;
    for (int it = 0; it < 4000; ++it) {
        const uint32_t n = it < 70 ? (uint32_t)it : (uint32_t)(g() % 2000);
        std::set<unsigned long long> ks;
        while (ks.size() < n) ks.insert(g() >> (g() % 40));
        std::vector<unsigned long long> key(ks.begin(), ks.end());
        std::shuffle(key.begin(), key.end(), g);
        std::vector<unsigned long long> kb(n + 2, guard);
        std::vector<float> wb(n + 2, -7.0f);
        for (uint32_t i = 0; i < n; ++i) {
            kb[i + 1] = key[i];
            wb[i + 1] = (float)(key[i] % 100003) * 0.5f;
        }
        sort_events(kb.data() + 1, wb.data() + 1, n);
        std::sort(key.begin(), key.end());
        if (kb[0] != guard || kb[n + 1] != guard || wb[0] != -7.0f || wb[n + 1] != -7.0f) {
            std::printf("write outside the range, case %d\n", it);
            return 1;
        }
        for (uint32_t i = 0; i < n; ++i)
            if (kb[i + 1] != key[i] || wb[i + 1] != (float)(key[i] % 100003) * 0.5f) {
                std::printf("case %d (n = %u): wrong at %u\n", it, n, i);
                return 1;
            }
    }
    std::printf("ok\n");
    return 0;
}
"""


def _kernel_sort_source():
    src = open(os.path.join(ROOT, "paper_1310_8478_amd", "csrc", "step.hip")).read()
    a = src.index("__device__ __forceinline__ void sift_events")
    b = src.index("template <uint32_t MODE>", a)
    code = src[a:b]
    assert "void sort_events" in code
    code = code.replace("__device__ __forceinline__", "static inline").replace("__restrict__", "")
    return "#include <cstdint>\n" + code


def _sanitizers_available(tmp_path):
    probe = tmp_path / "p.cpp"
    probe.write_text("int main() { return 0; }\n")
    r = subprocess.run(["g++", "-fsanitize=address,undefined", str(probe), "-o", str(tmp_path / "p")],
                       capture_output=True)
    return r.returncode == 0


def test_event_sort_against_std_sort(tmp_path):
    if subprocess.run(["g++", "--version"], capture_output=True).returncode != 0:
        pytest.skip("g++ not available")
    code = _kernel_sort_source()
    assert re.search(r"static inline void sort_events", code)
    cpp = tmp_path / "sort_check.cpp"
    cpp.write_text(code + DRIVER)
    flags = ["-O1", "-g", "-std=c++17"]
    if _sanitizers_available(tmp_path):
        flags += ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    exe = tmp_path / "sort_check"
    subprocess.check_call(["g++", *flags, str(cpp), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
    assert "runtime error" not in r.stderr, r.stderr
