"""Division by invariant integers of the outlier index kernel
(paper_2201_04614_amd/csrc/dq_fastdiv.hpp): the multiply-high form against
plain integer division, for every divisor below 20000 and random 32-bit
divisors (with random numerators, multiples of the divisor and their
neighbours, and the extremes), compiled for the host with hipcc."""

import os
import shutil
import subprocess

import pytest

CSRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2201_04614_amd", "csrc")

PROG = r"""
#include "dq_fastdiv.hpp"
#include <cstdio>
#include <random>
int main() {
    std::mt19937_64 g(7);
    long checked = 0, wrong = 0;
    auto check = [&](uint32_t d, uint32_t n) {
        const dq::FastDiv f = dq::make_fastdiv(d);
        ++checked;
        if (f.div(n) != n / d) {
            if (wrong < 5) printf("d=%u n=%u got %u\n", d, n, f.div(n));
            ++wrong;
        }
    };
    auto around_multiples = [&](uint32_t d) {
        for (uint64_t k = 1; k < 40; ++k) {
            const uint64_t v = k * (uint64_t)d;
            if (v > 0xffffffffull) break;
            check(d, (uint32_t)v);
            check(d, (uint32_t)(v - 1));
        }
    };
    for (uint32_t d = 1; d < 20000; ++d) {
        for (int k = 0; k < 60; ++k) check(d, (uint32_t)g());
        const uint32_t edge[] = {0u, 1u, d - 1, d, d + 1, 0x7fffffffu, 0x80000000u, 0xfffffffeu, 0xffffffffu};
        for (uint32_t n : edge) check(d, n);
        around_multiples(d);
    }
    for (int k = 0; k < 400000; ++k) {
        uint32_t d = (uint32_t)(g() >> (g() % 33));
        if (d == 0) d = 1;
        check(d, (uint32_t)g());
        check(d, 0xffffffffu);
        around_multiples(d);
    }
    for (int s = 0; s < 32; ++s)
        for (int k = 0; k < 1000; ++k) check(1u << s, (uint32_t)g());
    printf("%ld %ld\n", checked, wrong);
    return wrong != 0;
}
"""


def test_fastdiv_matches_integer_division(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc is not installed")
    src = tmp_path / "fastdiv_check.cpp"
    src.write_text(PROG)
    exe = tmp_path / "fastdiv_check"
    r = subprocess.run([hipcc, "--cuda-host-only", "-x", "hip", "-O2", "-std=c++17", "-I", CSRC, "-o", str(exe),
                        str(src)], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stdout[-2000:]
    checked, wrong = (int(v) for v in out.stdout.split()[-2:])
    assert wrong == 0 and checked > 1_000_000
