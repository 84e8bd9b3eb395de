"""The exponent map's division by multiply and shift, checked on the CPU.

The half-storage kernels find line q's exponent at (q mod m) a0 + (q div m) a1
+ ..., taking q div m as (q * qmul) >> qshift with the multiplier the host
computes (set_exp_qmod).  Granlund and Montgomery's theorem makes that exact
for every q < 2^31; this test compiles the host's own set_exp_qmod and checks
the product against integer division for many divisors and the quotient
boundaries of each.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2002_04896_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

PROGRAM = r"""
#include <cstdio>
#include <cstdint>
#include <vector>
#include "croft_internal.h"

using croft::ExpMap;

static uint64_t state = 0x9e3779b97f4a7c15ULL;
static uint64_t next() {  // splitmix64
    uint64_t z = (state += 0x9e3779b97f4a7c15ULL);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
    return z ^ (z >> 31);
}

int main() {
    const long long qlim = 1LL << 31;
    std::vector<long long> ds;
    for (long long d = 1; d <= 4096; ++d) ds.push_back(d);
    for (int k = 12; k <= 31; ++k) {
        ds.push_back(1LL << k);
        ds.push_back((1LL << k) - 1);
        ds.push_back((1LL << k) + 1);
    }
    for (int i = 0; i < 2000; ++i) ds.push_back(1 + (long long)(next() % (unsigned long long)qlim));
    long long checked = 0;
    for (long long d : ds) {
        if (d > qlim) continue;
        ExpMap m;
        croft::set_exp_qmod(m, d);
        if (m.qmod != d || m.qmul >= (1ULL << 32) || m.qshift < 31 || m.qshift > 62) {
            std::printf("bad multiplier for %lld: %llu >> %d\n", d, (unsigned long long)m.qmul, m.qshift);
            return 1;
        }
        std::vector<long long> qs = {0, 1, d - 1, d, d + 1, qlim - 1, qlim - 2, qlim - d};
        for (long long k = 1; k <= 64; ++k) {
            qs.push_back(k * d - 1);
            qs.push_back(k * d);
            qs.push_back((qlim / d - k) * d);
            qs.push_back((qlim / d - k) * d - 1);
        }
        for (int i = 0; i < 64; ++i) qs.push_back((long long)(next() % (unsigned long long)qlim));
        for (long long q : qs) {
            if (q < 0 || q >= qlim) continue;
            const unsigned long long got = ((unsigned long long)(unsigned)q * m.qmul) >> m.qshift;
            if ((long long)got != q / d) {
                std::printf("q %lld d %lld: %llu != %lld\n", q, d, got, q / d);
                return 1;
            }
            ++checked;
        }
    }
    std::printf("ok %lld\n", checked);
    return 0;
}
"""


def test_multiply_shift_matches_integer_division(tmp_path):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    src = tmp_path / "div.cpp"
    exe = tmp_path / "div"
    src.write_text(PROGRAM)
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", f"-I{CSRC}", str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok "), out.stdout
    assert int(out.stdout.split()[1]) > 1_000_000
