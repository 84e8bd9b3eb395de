"""The planner's host tables, checked on the CPU: the twiddle factors
w_n^m = exp(-2 pi i m / n) computed in FP64 and rounded once to FP32, and
Bluestein's chirp and kernel DFT.

The planner source (csrc/croft_plan.cpp) is compiled on its own into a small
shared library.  The references are independent of it: numpy's extended
precision (x87 80-bit long double) cos and sin, exact symmetries of the unit
circle, numpy's FFT (pocketfft) and, end to end, Bluestein's identity
DFT(x)[k] = c[k] sum_j x[j] c[j] conj(c[k - j]) evaluated with the tables and
compared with numpy's FFT of x.
"""
import ctypes
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2002_04896_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

WRAP = r"""
#include "croft_internal.h"
extern "C" {
void t_twiddles_fp64(int n, double *out) { croft::twiddles_fp64(n, out); }
void t_round_to_fp32(const double *in, size_t count, float *out) { croft::round_to_fp32(in, count, out); }
void t_bluestein(int n, int m, double *chirp, double *bhat) { croft::bluestein_tables_fp64(n, m, chirp, bhat); }
int t_bluestein_length(int n) { return croft::bluestein_length(n); }
}
"""


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    if not shutil.which(HIPCC) and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("tables")
    src = d / "wrap.cpp"
    so = d / "libtables.so"
    src.write_text(WRAP)
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", "-fPIC", "-shared", f"-I{CSRC}", str(src),
                        os.path.join(CSRC, "croft_plan.cpp"), "-o", str(so)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    L = ctypes.CDLL(str(so))
    dp = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
    fp = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
    L.t_twiddles_fp64.argtypes = [ctypes.c_int, dp]
    L.t_round_to_fp32.argtypes = [dp, ctypes.c_size_t, fp]
    L.t_bluestein.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
    L.t_bluestein_length.argtypes = [ctypes.c_int]
    L.t_bluestein_length.restype = ctypes.c_int
    return L


def twiddles(lib, n):
    out = np.empty(2 * n)
    lib.t_twiddles_fp64(n, out)
    return out[0::2] + 1j * out[1::2]


def exact_parts(n, m):
    """cos and -sin of 2 pi m / n in x87 extended precision (64-bit
    significand), the angle reduced exactly first: m mod n over n."""
    m = np.asarray(m, dtype=np.int64) % n
    two_pi = 2 * np.longdouble("3.14159265358979323846264338327950288")   # pi to the 64-bit significand
    ang = two_pi * m.astype(np.longdouble) / np.longdouble(n)
    return np.cos(ang), -np.sin(ang)


LENGTHS = [1, 2, 3, 4, 5, 6, 8, 12, 16, 48, 60, 64, 72, 80, 96, 100, 128, 384, 512, 1000, 1024, 2048, 4096,
           8192, 2 * 4093]


@pytest.mark.skipif(np.finfo(np.longdouble).nmant < 63, reason="needs x87 extended precision")
@pytest.mark.parametrize("n", LENGTHS)
def test_twiddles_within_an_ulp_of_the_exact_values(lib, n):
    w = twiddles(lib, n)
    c, s = exact_parts(n, np.arange(n))
    err = np.maximum(np.abs(w.real - c), np.abs(w.imag - s)).astype(np.float64)
    # within one ulp of 1 (|w| <= 1): libm on the folded angle plus the
    # rounding of the angle itself
    assert err.max() <= 2.0 ** -52, (n, err.max())


@pytest.mark.parametrize("n", [n for n in LENGTHS if n > 1])
def test_twiddle_symmetries_are_exact(lib, n):
    w = twiddles(lib, n)
    m = np.arange(1, n)
    assert w[0] == 1
    # w[n - m] = conj(w[m]), bit for bit
    assert np.array_equal(w[n - m], np.conj(w[m]))
    if n % 2 == 0:
        assert w[n // 2] == -1
        k = np.arange(n // 2)
        assert np.array_equal(w[n // 2 - k][1:], -np.conj(w[k])[1:])    # w[n/2 - m] = -conj w[m]
    if n % 4 == 0:
        assert w[n // 4] == -1j and w[3 * n // 4] == 1j
        k = np.arange(1, n // 4)
        # w[n/4 - m] = -i conj(w[m]): re = -im w[m], im = -re w[m]
        assert np.array_equal(w[n // 4 - k].real, -w[k].imag)
        assert np.array_equal(w[n // 4 - k].imag, -w[k].real)
    if n % 8 == 0:
        h = w[n // 8]
        assert h.real == -h.imag == np.sqrt(0.5)


@pytest.mark.skipif(np.finfo(np.longdouble).nmant < 63, reason="needs x87 extended precision")
@pytest.mark.parametrize("n", [3, 5, 48, 60, 100, 384, 512, 1000, 4096])
def test_fp32_tables_are_the_fp64_values_rounded_once(lib, n):
    w = np.empty(2 * n)
    lib.t_twiddles_fp64(n, w)
    f = np.empty(2 * n, np.float32)
    lib.t_round_to_fp32(w, 2 * n, f)
    assert np.array_equal(f, w.astype(np.float32))        # round to nearest even of the FP64 value
    c, s = exact_parts(n, np.arange(n))
    exact = np.empty(2 * n, np.longdouble)
    exact[0::2], exact[1::2] = c, s
    # and so within half an FP32 ulp of the exact value (plus the FP64 error)
    ulp = np.spacing(np.abs(f)).astype(np.longdouble)
    ulp[f == 0] = np.longdouble(2.0 ** -149)
    assert np.all(np.abs(f.astype(np.longdouble) - exact) <= ulp / 2 + np.longdouble(2.0 ** -53))


@pytest.mark.skipif(np.finfo(np.longdouble).nmant < 63, reason="needs x87 extended precision")
@pytest.mark.parametrize("n", [7, 11, 13, 97, 1009, 2039, 4093])
def test_bluestein_tables(lib, n):
    m = lib.t_bluestein_length(n)
    assert m >= 2 * n - 1 and m & (m - 1) == 0 and m < 4 * n
    chirp = np.empty(2 * n)
    bhat = np.empty(2 * m)
    lib.t_bluestein(n, m, chirp, bhat)
    c = chirp[0::2] + 1j * chirp[1::2]
    bh = bhat[0::2] + 1j * bhat[1::2]
    # chirp c[j] = exp(-pi i j^2 / n), from the exact residue j^2 mod 2n
    j = np.arange(n, dtype=np.int64)
    r = (j * j) % (2 * n)
    cr, ci = exact_parts(2 * n, r)
    err = np.maximum(np.abs(c.real - cr), np.abs(c.imag - ci)).astype(np.float64)
    assert err.max() <= 2.0 ** -52
    # kernel b[i] = b[m - i] = conj c[i] (i < n), zero elsewhere; bhat = FFT(b) / m
    b = np.zeros(m, complex)
    b[:n] = np.conj(c)
    b[m - n + 1:] = np.conj(c[1:][::-1])
    ref = np.fft.fft(b) / m
    assert np.abs(bh - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())
    # end to end: Bluestein's identity with these tables is the DFT
    rng = np.random.Generator(np.random.PCG64(n))
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    a = np.zeros(m, complex)
    a[:n] = x * c
    conv = np.fft.ifft(np.fft.fft(a) * bh * m)[:n]
    got = c * conv
    want = np.fft.fft(x)
    assert np.linalg.norm(got - want) / np.linalg.norm(want) <= 1e-13
