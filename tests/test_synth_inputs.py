"""Checks of the seeded input generators (CPU only)."""
import hashlib
import os
import subprocess
import sys

import numpy as np
import pytest

import oracle
from paper_2002_04896_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def m4_closed_form(u):
    """Piecewise cubic form of the order-4 cardinal B-spline on [0, 4)."""
    u = np.asarray(u, float)
    out = np.zeros_like(u)
    a = (u >= 0) & (u < 1); out[a] = u[a] ** 3 / 6
    b = (u >= 1) & (u < 2); out[b] = (-3 * u[b] ** 3 + 12 * u[b] ** 2 - 12 * u[b] + 4) / 6
    c = (u >= 2) & (u < 3); out[c] = (3 * u[c] ** 3 - 24 * u[c] ** 2 + 60 * u[c] - 44) / 6
    d = (u >= 3) & (u < 4); out[d] = (4 - u[d]) ** 3 / 6
    return out


def splitmix64(z):
    m = (1 << 64) - 1
    z = (z + 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def pme_reference(nx, ny, nz, seed):
    """Slow pure-Python spreading with the closed-form spline."""
    m = (1 << 64) - 1
    g = np.zeros((nz, ny, nx))
    nbx, nby, nbz = (nx + 3) // 4, (ny + 3) // 4, (nz + 3) // 4
    qtot = 0.0
    for bz in range(nbz):
        for by in range(nby):
            for bx in range(nbx):
                x0, y0, z0 = 4 * bx, 4 * by, 4 * bz
                dx, dy, dz = min(4, nx - x0), min(4, ny - y0), min(4, nz - z0)
                block = bx + nbx * (by + nby * bz)
                for c in range(dx * dy * dz):
                    key = (seed * 0x9E3779B97F4A7C15 + 4 * (block * 64 + c)) & m
                    u = [o + d * ((splitmix64((key + t) & m) >> 11) * 2.0 ** -53)
                         for t, (o, d) in enumerate(((x0, dx), (y0, dy), (z0, dz)))]
                    q = 1.0 if (splitmix64((key + 3) & m) >> 63) else -1.0
                    qtot += q
                    fl = [int(np.floor(v)) for v in u]
                    w = [m4_closed_form(np.array([v - f + t for t in range(4)]))
                         for v, f in zip(u, fl)]
                    for c2 in range(4):
                        for b2 in range(4):
                            for a2 in range(4):
                                g[(fl[2] - c2) % nz, (fl[1] - b2) % ny, (fl[0] - a2) % nx] += \
                                    q * w[2][c2] * w[1][b2] * w[0][a2]
    return g, qtot


@pytest.mark.parametrize("shape", [(8, 8, 8), (6, 5, 7), (12, 4, 10), (3, 2, 2)], ids=str)
def test_pme_matches_closed_form_spreading(shape):
    nx, ny, nz = shape
    g, q = synth.pme_grid(nx, ny, nz, seed=11)
    gr, qr = pme_reference(nx, ny, nz, seed=11)
    assert q == qr
    np.testing.assert_allclose(g, gr, rtol=0, atol=1e-13)


def test_pme_partition_of_unity_and_dc():
    g, q = synth.pme_grid(48, 60, 44, seed=3)
    assert abs(g.sum() - q) <= 1e-9 * g.size
    y = oracle.dft3d(g.astype(complex))
    assert abs(y[0, 0, 0] - q) <= 1e-8 * g.size          # DC = total charge
    neg = np.roll(y[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))
    assert oracle.rel_l2(neg, np.conj(y)) <= 1e-13       # real input -> Hermitian


def _grid_hash(threads):
    code = ("import hashlib; from paper_2002_04896_amd import synth; "
            "g, q = synth.pme_grid(40, 36, 28, seed=5); "
            "print(hashlib.sha256(g.tobytes()).hexdigest(), q)")
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    return subprocess.check_output([sys.executable, "-c", code], cwd=ROOT, env=env).decode()


def test_pme_independent_of_thread_count():
    assert _grid_hash(1) == _grid_hash(4) == _grid_hash(7)


def test_generators_are_seeded():
    a = synth.uniform_c((4, 5, 6), 1)
    assert np.array_equal(a, synth.uniform_c((4, 5, 6), 1))
    assert a.real.min() >= -1 and a.real.max() < 1 and a.imag.min() >= -1
    b = synth.normal_c((30, 20, 10), 2)
    assert np.array_equal(b, synth.normal_c((30, 20, 10), 2))
    assert abs(b.real.std() - 1) < 0.05 and abs(b.imag.mean()) < 0.05
    d = synth.batch_dims(4)
    assert d.shape == (64, 3) and np.array_equal(d, synth.batch_dims(4))
    assert set(np.unique(d)) <= set(synth.BATCH_LENGTHS)


@pytest.mark.parametrize("kind,bits", [("f16", 11), ("bf16", 8)])
def test_quantize_half_roundtrip(kind, bits):
    v = synth.normal_c((6, 7, 20), 9)
    v[2, 3] = 0                                          # an all-zero line
    data, e = synth.quantize_half(v, kind)
    assert data.shape == (6, 7, 20, 2) and data.dtype == np.uint16
    assert e.shape == (6, 7) and e.dtype == np.int8 and e[2, 3] == 0
    back = oracle.decode_half(data, e, kind, 0)
    peak = np.maximum(np.abs(v.real), np.abs(v.imag)).max(axis=2, keepdims=True)
    err = np.maximum(np.abs(back.real - v.real), np.abs(back.imag - v.imag))
    assert np.all(err <= peak * 2.0 ** -bits)


def test_pme_influence_is_even_finite_and_zero_at_dc():
    nx, ny, nz = 12, 10, 8
    g = synth.pme_influence(nx, ny, nz)
    assert g.shape == (nz, ny, nx // 2 + 1)
    assert np.all(np.isfinite(g)) and np.all(g >= 0) and g[0, 0, 0] == 0
    # G(-k) = G(k): mirror ky and kz
    mirror = g[(-np.arange(nz)) % nz][:, (-np.arange(ny)) % ny]
    np.testing.assert_allclose(g, mirror, rtol=1e-14, atol=0)
    # the B-spline modulus of the order-4 spline at the Nyquist frequency is 9
    # (1 / |1/6 - 2/3 + 1/6|^2), and the Gaussian decays away from k = 0
    assert g[0, 0, 1] > g[0, 0, 2] > g[0, 0, 3]
