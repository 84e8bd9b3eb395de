"""FP64 CPU oracle for the complex-to-complex 3D DFT -- TEST INFRASTRUCTURE.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never loads it, and it
shares no code with the GPU library.

What it computes (the paper, Section 2.1):

* ``dft3d(x, sign=-1)``  -- Eq. (1), the forward 3D DFT, as naive O(n^2) 1D DFTs
  along x, y, z (separability, Section 2.1), in C (``croft_oracle.c``).
* ``dft3d(x, sign=+1)``  -- the backward sum of Eq. (2) *without* its 1/N
  factor; ``backward_eq2`` divides by N and is Eq. (2) itself.
* ``dft3d_brute``        -- the triple sum of Eq. (1) evaluated directly.
* ``dft3d_lines``        -- exact output lines of large grids.
* ``dft_axis_lines``     -- the 1D transform of a range of lines along one axis
  (the building block of ``dft3d``; used to time a bounded sample).
* ``rdft3d``             -- forward transform of a real grid: Eq. (1) for
  kx = 0..nx/2 (the rest is fixed by Hermitian symmetry); ``rdft3d_lines``
  gives exact half-spectrum lines of large grids.
* ``irdft3d``            -- backward transform of a half spectrum to a real
  grid: the unnormalised backward sum over z and y, then the real inverse
  of the Hermitian extension along x (``c2r_x``); ``irdft3d_lines`` gives
  exact real output lines of large grids (``yz_sums`` + ``c2r_x``).
* ``convolve_real``      -- the reciprocal-space step of PME (Section 1): the
  forward real transform, a product with a real multiplier on the half
  spectrum, the backward real transform, and the sum of G |Q|^2 over the full
  spectrum.
* ``decode_half``        -- the exact value of FP16/BF16 storage with per-line
  power-of-two exponents (value = stored * 2**e).
* ``rel_l2``             -- the error metric ||a - ref||_2 / ||ref||_2.

Arrays have the numpy shape ``(nz, ny, nx)``: element (x, y, z) is at flat
index ``x + nx*(y + ny*z)``.

Every function is pinned by tests/test_oracle_pins.py against closed forms,
brute force and an independent library FFT.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "croft_oracle.c")
LIB = os.path.join(_HERE, "libcroft_oracle.so")
_lib = None

FORWARD = -1
BACKWARD = +1


def compile_oracle(src: str, out: str) -> str:
    """gcc -O2 with OpenMP; no fast-math, no FMA contraction."""
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                           "-ffp-contract=off", src, "-o", out, "-lm"])
    return out


def build() -> str:
    tmp = LIB + ".tmp"
    compile_oracle(SRC, tmp)
    os.replace(tmp, LIB)
    global _lib
    _lib = None
    return LIB


def bind(path: str):
    """Load an oracle shared library and declare its C signatures."""
    lib = ctypes.CDLL(path)
    i, l, p = ctypes.c_int, ctypes.c_long, ctypes.c_void_p
    lib.oracle_max_threads.argtypes = []
    lib.oracle_max_threads.restype = i
    lib.oracle_dft_axis_lines.argtypes = [i, i, i, p, i, l, l, i]
    lib.oracle_dft_axis_lines.restype = i
    lib.oracle_dft3d.argtypes = [i, i, i, p, i]
    lib.oracle_dft3d.restype = i
    lib.oracle_dft3d_zyx.argtypes = [i, i, i, p, i]
    lib.oracle_dft3d_zyx.restype = i
    lib.oracle_dft3d_brute.argtypes = [i, i, i, p, p, i]
    lib.oracle_dft3d_brute.restype = i
    lib.oracle_dft3d_lines.argtypes = [i, i, i, p, i, i, p, p, p]
    lib.oracle_dft3d_lines.restype = i
    lib.oracle_yz_sums.argtypes = [i, i, i, p, i, i, p, p, p]
    lib.oracle_yz_sums.restype = i
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: run __graft_entry__.build() first")
        _lib = bind(LIB)
    return _lib


class Oracle:
    """The oracle's entry points over one loaded library (the default one, or
    another build of the same source, e.g. a deliberately mutated copy)."""

    def __init__(self, lib=None):
        self.lib = lib if lib is not None else _load()

    @staticmethod
    def _grid(x) -> np.ndarray:
        a = np.ascontiguousarray(np.asarray(x), dtype=np.complex128)
        if a.ndim != 3:
            raise ValueError("expected a (nz, ny, nx) array")
        return a

    def max_threads(self) -> int:
        return int(self.lib.oracle_max_threads())

    def dft3d(self, x, sign: int = FORWARD) -> np.ndarray:
        a = self._grid(x).copy()
        nz, ny, nx = a.shape
        if self.lib.oracle_dft3d(nx, ny, nz, a.ctypes.data, sign) != 0:
            raise ValueError("oracle_dft3d failed")
        return a

    def dft3d_zyx(self, x, sign: int = FORWARD) -> np.ndarray:
        a = self._grid(x).copy()
        nz, ny, nx = a.shape
        if self.lib.oracle_dft3d_zyx(nx, ny, nz, a.ctypes.data, sign) != 0:
            raise ValueError("oracle_dft3d_zyx failed")
        return a

    def dft3d_brute(self, x, sign: int = FORWARD) -> np.ndarray:
        a = self._grid(x)
        out = np.empty_like(a)
        nz, ny, nx = a.shape
        if self.lib.oracle_dft3d_brute(nx, ny, nz, a.ctypes.data, out.ctypes.data, sign) != 0:
            raise ValueError("oracle_dft3d_brute failed")
        return out

    def dft3d_lines(self, x, kyz, sign: int = FORWARD) -> np.ndarray:
        """Y(kx, ky, kz) for all kx and each (ky, kz) in ``kyz``: (len(kyz), nx)."""
        a = self._grid(x)
        nz, ny, nx = a.shape
        kyz = np.asarray(kyz, dtype=np.int32).reshape(-1, 2)
        ky = np.ascontiguousarray(kyz[:, 0])
        kz = np.ascontiguousarray(kyz[:, 1])
        out = np.empty((len(kyz), nx), dtype=np.complex128)
        rc = self.lib.oracle_dft3d_lines(nx, ny, nz, a.ctypes.data, sign, len(kyz),
                                         ky.ctypes.data, kz.ctypes.data, out.ctypes.data)
        if rc != 0:
            raise ValueError("oracle_dft3d_lines failed")
        return out

    def yz_sums(self, x, kyz, sign: int = FORWARD) -> np.ndarray:
        """For each (ky, kz) in ``kyz`` and every x: the y and z sums of the
        transform with the given sign, before any sum over x: (len(kyz), nx)."""
        a = self._grid(x)
        nz, ny, nx = a.shape
        kyz = np.asarray(kyz, dtype=np.int32).reshape(-1, 2)
        ky = np.ascontiguousarray(kyz[:, 0])
        kz = np.ascontiguousarray(kyz[:, 1])
        out = np.empty((len(kyz), nx), dtype=np.complex128)
        rc = self.lib.oracle_yz_sums(nx, ny, nz, a.ctypes.data, sign, len(kyz),
                                     ky.ctypes.data, kz.ctypes.data, out.ctypes.data)
        if rc != 0:
            raise ValueError("oracle_yz_sums failed")
        return out

    def dft_axis_lines(self, a: np.ndarray, axis: int, first: int, count: int,
                       sign: int = FORWARD) -> None:
        """In place on a C-contiguous complex128 (nz, ny, nx) array."""
        if a.dtype != np.complex128 or not a.flags.c_contiguous or a.ndim != 3:
            raise ValueError("need a C-contiguous complex128 (nz, ny, nx) array")
        nz, ny, nx = a.shape
        if self.lib.oracle_dft_axis_lines(nx, ny, nz, a.ctypes.data, axis, first, count,
                                          sign) != 0:
            raise ValueError("oracle_dft_axis_lines failed")


_default = None


def _o() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle()
    return _default


def max_threads() -> int:
    return _o().max_threads()


def dft3d(x, sign: int = FORWARD) -> np.ndarray:
    """Eq. (1) for sign -1; the unnormalised backward sum of Eq. (2) for +1."""
    return _o().dft3d(x, sign)


def dft3d_zyx(x, sign: int = FORWARD) -> np.ndarray:
    return _o().dft3d_zyx(x, sign)


def dft3d_brute(x, sign: int = FORWARD) -> np.ndarray:
    return _o().dft3d_brute(x, sign)


def dft3d_lines(x, kyz, sign: int = FORWARD) -> np.ndarray:
    return _o().dft3d_lines(x, kyz, sign)


def dft_axis_lines(a, axis, first, count, sign: int = FORWARD) -> None:
    _o().dft_axis_lines(a, axis, first, count, sign)


def yz_sums(x, kyz, sign: int = FORWARD) -> np.ndarray:
    return _o().yz_sums(x, kyz, sign)


# ------------------------------------------------------------ real transforms
# The PME charge grid of Section 1 is real; the spectrum of a real grid obeys
# Y(-k) = conj Y(k) under Eq. (1), so its kx = 0..nx/2 half holds everything.

def rdft3d(x) -> np.ndarray:
    """Eq. (1) of a real (nz, ny, nx) grid, kept for kx = 0..nx/2:
    shape (nz, ny, nx//2 + 1)."""
    a = np.asarray(x, dtype=np.float64)
    if a.ndim != 3:
        raise ValueError("expected a real (nz, ny, nx) array")
    return np.ascontiguousarray(dft3d(a.astype(np.complex128), FORWARD)[:, :, : a.shape[2] // 2 + 1])


def rdft3d_lines(x, kyz) -> np.ndarray:
    """Half-spectrum lines Y(0..nx/2, ky, kz) of a real grid: (len(kyz), nx//2 + 1)."""
    a = np.asarray(x, dtype=np.float64)
    return dft3d_lines(a.astype(np.complex128), kyz, FORWARD)[:, : a.shape[2] // 2 + 1]


def c2r_x(g, nx: int) -> np.ndarray:
    """Real inverse along x of half-spectrum lines g[..., 0..nx/2] (nx even),
    unnormalised: the sum over kx = 0..nx-1 of the Hermitian extension
    G(nx - k) = conj G(k), times exp(+2 pi i k n / nx).  Written out, with
    m = nx/2 (the imaginary parts of G(0) and G(m) drop out of the sum):
        x(n) = Re G(0) + (-1)^n Re G(m) + 2 Re sum_{0<k<m} G(k) exp(2 pi i k n / nx).
    """
    g = np.asarray(g, dtype=np.complex128)
    if nx % 2 or g.shape[-1] != nx // 2 + 1:
        raise ValueError("need nx even and nx//2 + 1 values per line")
    m = nx // 2
    n = np.arange(nx)
    k = np.arange(1, m)
    phase = 2.0 * np.pi * ((k[:, None] * n[None, :]) % nx) / nx   # exact k n mod nx
    e = np.cos(phase) + 1j * np.sin(phase)
    sign_n = np.where(n % 2 == 0, 1.0, -1.0)
    inner = g[..., 1:m] @ e if m > 1 else np.zeros(g.shape[:-1] + (nx,), np.complex128)
    return g[..., :1].real + sign_n * g[..., m:m + 1].real + 2.0 * inner.real


def irdft3d(h, nx: int) -> np.ndarray:
    """Backward transform of a half spectrum h (nz, ny, nx//2 + 1) to a real
    (nz, ny, nx) grid, without Eq. (2)'s 1/N: the backward sums along z and y
    (sign +1), then ``c2r_x`` along x.  For the half spectrum of a real grid
    this is N times that grid."""
    a = np.ascontiguousarray(np.asarray(h), dtype=np.complex128).copy()
    if a.ndim != 3:
        raise ValueError("expected a (nz, ny, nx//2 + 1) array")
    nz, ny, hx = a.shape
    dft_axis_lines(a, 1, 0, hx * nz, BACKWARD)
    dft_axis_lines(a, 2, 0, hx * ny, BACKWARD)
    return c2r_x(a, nx)


def irdft3d_lines(h, nx: int, yz) -> np.ndarray:
    """Real output lines x(0..nx-1, y, z) of ``irdft3d`` for each (y, z) in
    ``yz``: (len(yz), nx)."""
    return c2r_x(yz_sums(h, yz, BACKWARD), nx)


def half_weights(nx: int) -> np.ndarray:
    """How many full-spectrum bins each kx = 0..nx/2 of a half spectrum
    stands for: 1 for kx = 0 and kx = nx/2, 2 for the rest (their mirrors
    nx - kx hold the conjugate values)."""
    w = np.full(nx // 2 + 1, 2.0)
    w[0] = 1.0
    w[nx // 2] = 1.0
    return w


def convolve_real(x, g):
    """PME's reciprocal-space step on a real (nz, ny, nx) grid with a real
    multiplier g on the half spectrum (nz, ny, nx//2 + 1):
        Q = rdft3d(x)                      (Eq. 1, kx <= nx/2)
        out = irdft3d(g * Q, nx)           (backward, no 1/N)
        energy = sum over the full spectrum of G |Q|^2, G(-k) = G(k),
               = sum over the half of half_weights(nx) * g * |Q|^2.
    Returns (out, energy)."""
    a = np.asarray(x, dtype=np.float64)
    gg = np.asarray(g, dtype=np.float64)
    nx = a.shape[2]
    q = rdft3d(a)
    if gg.shape != q.shape:
        raise ValueError("multiplier must have the half-spectrum shape (nz, ny, nx//2 + 1)")
    out = irdft3d(gg * q, nx)
    energy = float(np.sum(half_weights(nx) * gg * (q.real ** 2 + q.imag ** 2)))
    return out, energy


def backward_eq2(y) -> np.ndarray:
    """Eq. (2): the backward sum scaled by 1/(Nx Ny Nz)."""
    a = dft3d(y, BACKWARD)
    return a / a.size


def decode_half(data, exp, kind: str, line_axis: int) -> np.ndarray:
    """Exact complex128 value of 16-bit storage with per-line exponents.

    ``data``: uint16 (or float16/bfloat16 bit patterns) of shape (nz, ny, nx, 2)
    holding (re, im); ``kind`` is "f16" (IEEE binary16) or "bf16" (bfloat16,
    the upper half of an IEEE binary32).  ``exp``: int8, one per line along
    ``line_axis`` -- shape (nz, ny) for x-lines (axis 0), (nz, nx) for y-lines
    (axis 1), (ny, nx) for z-lines (axis 2).  Value = stored * 2**exp, exact.
    """
    bits = np.ascontiguousarray(np.asarray(data)).view(np.uint16)
    if kind == "f16":
        parts = bits.view(np.float16).astype(np.float64)
    elif kind == "bf16":
        parts = (bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    else:
        raise ValueError(kind)
    e = np.asarray(exp).astype(np.int64)
    if line_axis == 0:
        e = e[:, :, None]
    elif line_axis == 1:
        e = e[:, None, :]
    elif line_axis == 2:
        e = e[None, :, :]
    else:
        raise ValueError(line_axis)
    val = parts[..., 0] + 1j * parts[..., 1]
    return np.ldexp(val.real, e) + 1j * np.ldexp(val.imag, e)


def rel_l2(a, ref) -> float:
    """||a - ref||_2 / ||ref||_2 over all real and imaginary components (FP64);
    the absolute ||a||_2 when ref is all zero."""
    a = np.asarray(a, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    den = float(np.sqrt(np.sum(np.abs(ref) ** 2)))
    num = float(np.sqrt(np.sum(np.abs(a - ref) ** 2)))
    return num / den if den > 0 else num
