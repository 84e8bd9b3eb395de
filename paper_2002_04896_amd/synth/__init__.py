"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws input values; it holds no part of the transform itself.
Both the GPU path and the CPU oracle receive the arrays it returns.

Inputs (the paper benchmarks double-complex grids of 128^3 and 1024^3 with no
stated values, Section 6.1.2; the grids below stand in for them):

* ``uniform_c``  -- real and imaginary parts iid Uniform[-1, 1), numpy PCG64.
* ``normal_c``   -- real and imaginary parts iid N(0, 1), numpy PCG64.
* ``pme_grid``   -- charges +-1 spread by the order-4 cardinal B-spline onto a
  periodic grid, one charge per cell on average (particle-mesh Ewald, the
  paper's motivating application, Section 1); real valued.  Built by the C
  helper ``pme_spread.c`` (counter-based RNG, thread-count independent).
* ``pme_influence`` -- the smooth-PME reciprocal-space multiplier on the half
  spectrum (Gaussian-screened Coulomb kernel times the order-4 B-spline
  moduli, Essmann et al. 1995), the real multiplier of a convolution plan.
* ``batch_dims`` -- the uneven shapes of a batch of grids.
* ``quantize_half`` -- an input encoded as FP16/BF16 pairs with one
  power-of-two exponent per x-line (value = stored * 2**e).

Arrays use the torch/numpy shape ``(nz, ny, nx)``: element (x, y, z) sits at
flat index ``x + nx*(y + ny*z)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pme_spread.c")
_LIB = os.path.join(_HERE, "libcroft_synth.so")
_lib = None

BATCH_LENGTHS = (48, 60, 64, 72, 80, 96, 100, 128)


def build() -> str:
    """Compile the C helper in place (gcc, OpenMP). Returns the library path."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                           "-ffp-contract=off", _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    global _lib
    _lib = None
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise RuntimeError(f"{_LIB} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(_LIB)
        lib.synth_pme_spread.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                         ctypes.c_uint64, ctypes.c_void_p,
                                         ctypes.POINTER(ctypes.c_double)]
        lib.synth_pme_spread.restype = ctypes.c_int
        _lib = lib
    return _lib


def uniform_c(shape, seed: int) -> np.ndarray:
    """complex128 array, re and im iid Uniform[-1, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.uniform(-1.0, 1.0, size=shape)
    im = rng.uniform(-1.0, 1.0, size=shape)
    return re + 1j * im


def normal_c(shape, seed: int) -> np.ndarray:
    """complex128 array, re and im iid N(0, 1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.empty(shape, dtype=np.complex128)
    flat = out.reshape(-1).view(np.float64)
    rng.standard_normal(out=flat)  # interleaved re/im, all iid
    return out


def pme_grid(nx: int, ny: int, nz: int, seed: int):
    """Real PME charge grid of shape (nz, ny, nx) (float64) and the total charge."""
    lib = _load()
    grid = np.empty((nz, ny, nx), dtype=np.float64)
    q = ctypes.c_double(0.0)
    rc = lib.synth_pme_spread(nx, ny, nz, ctypes.c_uint64(seed), grid.ctypes.data,
                              ctypes.byref(q))
    if rc != 0:
        raise ValueError(f"bad PME grid size {(nx, ny, nz)}")
    return grid, q.value


def pme_influence(nx: int, ny: int, nz: int, beta: float = 0.3) -> np.ndarray:
    """Multiplier G on the half spectrum, shape (nz, ny, nx//2 + 1), float64.

    Unit grid spacing (box nx x ny x nz, volume V), Ewald parameter beta (per
    grid spacing).  For the reciprocal vector with components m_a / n_a
    (m_a the signed frequency of bin k_a):
        G = exp(-pi^2 |m|^2 / beta^2) / (pi V |m|^2) * B_x B_y B_z,   G(0) = 0,
    with the order-4 B-spline moduli B_a(k) = 1 / |sum_{j=0..2} M4(j+1)
    exp(2 pi i k j / n_a)|^2, M4(1) = M4(3) = 1/6, M4(2) = 2/3.
    """
    def signed(n, count):
        k = np.arange(count)
        return np.where(k <= n // 2, k, k - n) / n

    def bmod(n, count):
        k = np.arange(count)
        c = np.array([1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0])
        ph = 2.0 * np.pi * np.outer(k, np.arange(3)) / n
        s = (c * np.exp(1j * ph)).sum(axis=1)
        return 1.0 / np.abs(s) ** 2

    hx = nx // 2 + 1
    mx, my, mz = signed(nx, hx), signed(ny, ny), signed(nz, nz)
    m2 = mz[:, None, None] ** 2 + my[None, :, None] ** 2 + mx[None, None, :] ** 2
    with np.errstate(divide="ignore", invalid="ignore"):
        g = np.exp(-np.pi ** 2 * m2 / beta ** 2) / (np.pi * nx * ny * nz * m2)
    g[0, 0, 0] = 0.0
    return g * (bmod(nz, nz)[:, None, None] * bmod(ny, ny)[None, :, None] * bmod(nx, hx)[None, None, :])


def batch_dims(seed: int, count: int = 64, lengths=BATCH_LENGTHS) -> np.ndarray:
    """count x 3 array of (nx, ny, nz), each axis drawn from ``lengths``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.choice(np.asarray(lengths, dtype=np.int64), size=(count, 3))


def quantize_half(values: np.ndarray, kind: str):
    """Encode complex values (shape (nz, ny, nx)) as 16-bit pairs plus one int8
    exponent per x-line.

    Returns ``(data, exp)``: ``data`` is uint16 of shape (nz, ny, nx, 2) holding
    IEEE binary16 (kind "f16") or bfloat16 (kind "bf16") bit patterns of
    (re, im); ``exp`` is int8 of shape (nz, ny).  The represented value is
    ``stored * 2**exp``.  The exponent puts the largest |re|, |im| of each line
    just under 2**12; values are rounded to nearest even.
    """
    v = np.asarray(values, dtype=np.complex128)
    nz, ny, nx = v.shape
    parts = np.stack([v.real, v.imag], axis=-1)                 # (nz, ny, nx, 2)
    peak = np.abs(parts).max(axis=(2, 3))                       # (nz, ny)
    e = np.zeros((nz, ny), dtype=np.int64)
    nzero = peak > 0
    e[nzero] = np.ceil(np.log2(peak[nzero])).astype(np.int64) - 12
    e = np.clip(e, -128, 127)
    scaled = np.ldexp(parts, -e[:, :, None, None])
    if kind == "f16":
        data = scaled.astype(np.float16).view(np.uint16)
    elif kind == "bf16":
        f32 = scaled.astype(np.float32)
        bits = f32.view(np.uint32).astype(np.uint64)
        # round to nearest even on the upper 16 bits
        rounded = (bits + 0x7FFF + ((bits >> 16) & 1)) >> 16
        data = rounded.astype(np.uint16)
    else:
        raise ValueError(kind)
    return np.ascontiguousarray(data), e.astype(np.int8)
