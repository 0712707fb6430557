"""The sorts of the HIP path compiled for the host from the kernel source
itself and checked against std::sort, built with AddressSanitizer and
UndefinedBehaviorSanitizer where gcc has them:

* the in-place heapsort of the ORDERED fold (sift_events / sort_events in
  step.hip): random distinct keys of 0 .. 2000 events, weights moving with
  their keys, nothing written outside the range;
* the wavefront bitonic sort of the ORDERED fold (wave_sort_load /
  bitonic_stage in step.hip), run lane by lane for the 64 lanes between
  stages: 33 .. 1024 events, padding above every key, weights with keys;
* the bitonic network of the build's reverse-row sort (bitonic in
  build.hip), run by one host thread: rows of 2 .. 8192 entries."""
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


WAVE_DRIVER = r"""
#include <algorithm>
#include <cstdio>
#include <random>
#include <set>
#include <vector>
int main() {
    std::mt19937_64 g(11);
    const unsigned long long guard = 0x5555555555555555ull;
    const uint32_t cap = 1024;
    for (int it = 0; it < 3000; ++it) {
        const uint32_t fixed[] = {33, 63, 64, 65, 127, 128, 129, 1023, 1024};
        const uint32_t n = it < 9 ? fixed[it] : 33u + (uint32_t)(g() % 992);
        std::set<unsigned long long> ks;
        while (ks.size() < n) ks.insert((g() >> (g() % 30)) & ~(1ull << 63));
        std::vector<unsigned long long> key(ks.begin(), ks.end());
        std::shuffle(key.begin(), key.end(), g);
        std::vector<float> wt(n);
        for (uint32_t i = 0; i < n; ++i) wt[i] = (float)(key[i] % 100003) * 0.25f;
        std::vector<unsigned long long> sk(cap + 2, guard);
        std::vector<float> sw(cap + 2, -3.0f);
        uint32_t P = 0;
        for (uint32_t lane = 0; lane < 64; ++lane)
            P = wave_sort_load(key.data(), wt.data(), n, sk.data() + 1, sw.data() + 1, lane);
        for (uint32_t k = 2; k <= P; k <<= 1)
            for (uint32_t j = k >> 1; j > 0; j >>= 1)
                for (uint32_t lane = 0; lane < 64; ++lane)
                    bitonic_stage(sk.data() + 1, sw.data() + 1, P, k, j, lane);
        std::vector<unsigned long long> want(key);
        std::sort(want.begin(), want.end());
        if (P < n || P > cap || (P & (P - 1)) || sk[0] != guard || sk[cap + 1] != guard ||
            sw[0] != -3.0f || sw[cap + 1] != -3.0f) {
            std::printf("case %d: padding or bounds\n", it);
            return 1;
        }
        for (uint32_t x = P; x < cap; ++x)
            if (sk[x + 1] != guard) { std::printf("case %d: write past P\n", it); return 1; }
        for (uint32_t i = 0; i < P; ++i) {
            const unsigned long long k = sk[i + 1];
            if (i < n ? (k != want[i] || sw[i + 1] != (float)(want[i] % 100003) * 0.25f) : k != ~0ull) {
                std::printf("case %d (n = %u): wrong at %u\n", it, n, i);
                return 1;
            }
        }
    }
    std::printf("ok\n");
    return 0;
}
"""

ROW_DRIVER = r"""
#include <algorithm>
#include <cstdio>
#include <random>
#include <set>
#include <vector>
int main() {
    std::mt19937_64 g(13);
    for (int it = 0; it < 600; ++it) {
        const uint32_t n = it < 40 ? (uint32_t)(2 + it) : 2u + (uint32_t)(g() % 8191);
        std::set<unsigned long long> ks;
        while (ks.size() < n) ks.insert(g() % ((n < 200 ? 1000ull : 1ull << 62)));
        std::vector<unsigned long long> key(ks.begin(), ks.end());
        std::shuffle(key.begin(), key.end(), g);
        uint32_t P = 2;
        while (P < n) P <<= 1;
        std::vector<unsigned long long> sk(P + 2, 0x7777ull);
        for (uint32_t x = 0; x < P; ++x) sk[x + 1] = x < n ? key[x] : ~0ull;
        bitonic(sk.data() + 1, P, 0u, 1u, [] {});
        std::sort(key.begin(), key.end());
        if (sk[0] != 0x7777ull || sk[P + 1] != 0x7777ull) { std::printf("bounds %d\n", it); return 1; }
        for (uint32_t i = 0; i < P; ++i)
            if (sk[i + 1] != (i < n ? key[i] : ~0ull)) {
                std::printf("case %d (n = %u): wrong at %u\n", it, n, i);
                return 1;
            }
    }
    std::printf("ok\n");
    return 0;
}
"""


def _extract(fname, start, end):
    src = open(os.path.join(ROOT, "paper_1310_8478_amd", "csrc", fname)).read()
    a = src.index(start)
    b = src.index(end, a)
    code = src[a:b].replace("__device__ __forceinline__", "static inline").replace("__restrict__", "")
    return "#include <cstdint>\n" + code


def _run(tmp_path, name, code):
    if subprocess.run(["g++", "--version"], capture_output=True).returncode != 0:
        pytest.skip("g++ not available")
    cpp = tmp_path / f"{name}.cpp"
    cpp.write_text(code)
    flags = ["-O1", "-g", "-std=c++17"]
    if _sanitizers_available(tmp_path):
        flags += ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    exe = tmp_path / name
    subprocess.check_call(["g++", *flags, str(cpp), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=0"))
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
    assert "runtime error" not in r.stderr, r.stderr


def test_wave_bitonic_against_std_sort(tmp_path):
    code = _extract("step.hip", "__device__ __forceinline__ uint32_t wave_sort_load",
                    "// One target's n (kSelectFold")
    assert "static inline void bitonic_stage" in code
    _run(tmp_path, "wave_sort", code + WAVE_DRIVER)


def test_row_bitonic_against_std_sort(tmp_path):
    code = _extract("build.hip", "template <typename Sync>", "// Rows of 2 .. kSortShort")
    assert "void bitonic" in code
    _run(tmp_path, "row_sort", code + ROW_DRIVER)
