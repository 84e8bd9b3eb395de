"""Pins for the FP64 CPU oracle (no GPU).

Each test ties the oracle to something other than itself: values worked by
hand from Eq. (1)/(2) of the paper (tests/golden/), closed forms of the DFT,
invariants, the direct triple sum, and numpy's independent FFT (pocketfft).
"""
import glob
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.Generator(np.random.PCG64(12345))


def rand_grid(nz, ny, nx, rng=RNG):
    return rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))


def read_golden(path):
    shape = sign = None
    section = None
    vals = {"input": [], "output": []}
    with open(path) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "shape":
                shape = tuple(int(t) for t in tok[1:4])
            elif tok[0] == "sign":
                sign = int(tok[1])
            elif tok[0] in vals:
                section = tok[0]
            else:
                vals[section].append(float(tok[0]) + 1j * float(tok[1]))
    nx, ny, nz = shape
    x = np.array(vals["input"]).reshape(nz, ny, nx)
    y = np.array(vals["output"]).reshape(nz, ny, nx)
    return x, y, sign


GOLDEN_FILES = sorted(glob.glob(os.path.join(GOLDEN, "*.txt")))


@pytest.mark.parametrize("path", GOLDEN_FILES, ids=os.path.basename)
def test_golden_worked_examples(path):
    x, y, sign = read_golden(path)
    for got in (oracle.dft3d(x, sign), oracle.dft3d_brute(x, sign), oracle.dft3d_zyx(x, sign)):
        np.testing.assert_allclose(got, y, rtol=0, atol=1e-13 * max(1.0, np.abs(y).max()))


def test_golden_files_present():
    assert len(GOLDEN_FILES) >= 5


TINY = [(2, 3, 5), (8, 6, 4), (5, 5, 5), (7, 1, 3), (8, 8, 8), (1, 1, 1), (3, 4, 1), (1, 9, 2)]


@pytest.mark.parametrize("nxyz", TINY, ids=str)
@pytest.mark.parametrize("sign", [-1, 1])
def test_separable_equals_brute_force(nxyz, sign):
    nx, ny, nz = nxyz
    x = rand_grid(nz, ny, nx)
    ref = oracle.dft3d_brute(x, sign)
    assert oracle.rel_l2(oracle.dft3d(x, sign), ref) <= 1e-13
    assert oracle.rel_l2(oracle.dft3d_zyx(x, sign), ref) <= 1e-13


NUMPY_SHAPES = [(32, 32, 32), (48, 60, 100), (1, 1, 7), (64, 16, 4), (27, 25, 16),
                (5, 128, 3), (100, 48, 60)]


@pytest.mark.parametrize("nzyx", NUMPY_SHAPES, ids=str)
def test_matches_numpy_pocketfft(nzyx):
    x = rand_grid(*nzyx)
    assert oracle.rel_l2(oracle.dft3d(x, -1), np.fft.fftn(x)) <= 1e-12
    assert oracle.rel_l2(oracle.dft3d(x, +1), np.fft.ifftn(x) * x.size) <= 1e-12
    assert oracle.rel_l2(oracle.backward_eq2(x), np.fft.ifftn(x)) <= 1e-12


def test_delta_at_origin_gives_ones():
    x = np.zeros((6, 10, 12), complex)
    x[0, 0, 0] = 1
    np.testing.assert_allclose(oracle.dft3d(x), np.ones_like(x), atol=1e-14)


@pytest.mark.parametrize("sign", [-1, 1])
def test_shifted_delta_gives_plane_wave(sign):
    # asymmetric shift on a non-cubic grid pins the sign, the twiddles and the
    # mapping between axes and strides
    nx, ny, nz = 12, 10, 6
    ax, ay, az = 5, 3, 1
    x = np.zeros((nz, ny, nx), complex)
    x[az, ay, ax] = 1
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    want = np.exp(sign * 2j * np.pi * (kx * ax / nx + ky * ay / ny + kz * az / nz))
    np.testing.assert_allclose(oracle.dft3d(x, sign), want, atol=1e-13)


def test_plane_wave_gives_spike():
    nx, ny, nz = 20, 9, 8
    mx, my, mz = 7, 2, 5
    jz, jy, jx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    x = np.exp(2j * np.pi * (mx * jx / nx + my * jy / ny + mz * jz / nz))
    want = np.zeros_like(x)
    want[mz, my, mx] = x.size
    np.testing.assert_allclose(oracle.dft3d(x), want, atol=1e-10)


def test_constant_gives_dc_spike():
    x = np.full((5, 4, 3), 2.5 - 1j)
    want = np.zeros_like(x)
    want[0, 0, 0] = x.size * (2.5 - 1j)
    np.testing.assert_allclose(oracle.dft3d(x), want, atol=1e-12)


def test_linearity():
    a, b = rand_grid(8, 12, 10), rand_grid(8, 12, 10)
    al, be = 0.7 - 1.3j, -2.1 + 0.4j
    lhs = oracle.dft3d(al * a + be * b)
    rhs = al * oracle.dft3d(a) + be * oracle.dft3d(b)
    assert oracle.rel_l2(lhs, rhs) <= 1e-13


def test_parseval():
    x = rand_grid(9, 16, 20)
    y = oracle.dft3d(x)
    assert abs(np.sum(np.abs(y) ** 2) - x.size * np.sum(np.abs(x) ** 2)) \
        <= 1e-12 * x.size * np.sum(np.abs(x) ** 2)


def test_forward_then_backward_is_n_identity():
    x = rand_grid(10, 6, 15)
    back = oracle.dft3d(oracle.dft3d(x, -1), +1)
    assert oracle.rel_l2(back, x.size * x) <= 1e-13


def test_circular_shift_gives_phase_ramp():
    nx, ny, nz = 16, 15, 10
    sx, sy, sz = 3, 7, 4
    x = rand_grid(nz, ny, nx)
    shifted = np.roll(x, (sz, sy, sx), axis=(0, 1, 2))
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ramp = np.exp(-2j * np.pi * (kx * sx / nx + ky * sy / ny + kz * sz / nz))
    assert oracle.rel_l2(oracle.dft3d(shifted), ramp * oracle.dft3d(x)) <= 1e-13


def test_separable_product_gives_product_of_1d_dfts():
    nx, ny, nz = 24, 10, 9
    fx = RNG.standard_normal(nx) + 1j * RNG.standard_normal(nx)
    fy = RNG.standard_normal(ny) + 1j * RNG.standard_normal(ny)
    fz = RNG.standard_normal(nz) + 1j * RNG.standard_normal(nz)
    x = fz[:, None, None] * fy[None, :, None] * fx[None, None, :]
    want = (np.fft.fft(fz)[:, None, None] * np.fft.fft(fy)[None, :, None]
            * np.fft.fft(fx)[None, None, :])
    assert oracle.rel_l2(oracle.dft3d(x), want) <= 1e-13


def test_real_input_gives_hermitian_output():
    x = RNG.standard_normal((8, 10, 12)).astype(complex)
    y = oracle.dft3d(x)
    neg = np.roll(y[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))      # Y(-k)
    assert oracle.rel_l2(neg, np.conj(y)) <= 1e-13


def test_exact_lines_match_full_transform():
    x = rand_grid(30, 20, 24)
    full = oracle.dft3d(x)
    kyz = [(0, 0), (3, 7), (19, 29), (10, 1)]
    for sign, ref in ((-1, full), (+1, oracle.dft3d(x, +1))):
        lines = oracle.dft3d_lines(x, kyz, sign)
        for i, (ky, kz) in enumerate(kyz):
            assert oracle.rel_l2(lines[i], ref[kz, ky, :]) <= 1e-13


def test_axis_line_range_transforms_only_those_lines():
    x = rand_grid(6, 10, 8)
    a = x.copy()
    # y-lines are numbered l = x + nx*z; take lines 5 .. 5+17
    oracle.dft_axis_lines(a, 1, 5, 17)
    want = x.copy()
    for l in range(5, 22):
        xi, zi = l % 8, l // 8
        want[zi, :, xi] = np.fft.fft(x[zi, :, xi])
    assert oracle.rel_l2(a, want) <= 1e-13
    b = x.copy()
    oracle.dft_axis_lines(b, 2, 0, 80)                    # every z-line
    assert oracle.rel_l2(b, np.fft.fft(x, axis=0)) <= 1e-13
    c = x.copy()
    oracle.dft_axis_lines(c, 0, 0, 60)                    # every x-line
    assert oracle.rel_l2(c, np.fft.fft(x, axis=2)) <= 1e-13


def test_oracle_rejects_bad_arguments():
    with pytest.raises(ValueError):
        oracle.dft3d(np.zeros((2, 2)))
    with pytest.raises(ValueError):
        oracle.dft_axis_lines(np.zeros((2, 2, 2), complex), 3, 0, 1)
    with pytest.raises(ValueError):
        oracle.dft_axis_lines(np.zeros((2, 2, 2), complex), 0, 3, 2)
    with pytest.raises(ValueError):
        oracle.dft3d_lines(np.zeros((2, 2, 2), complex), [(2, 0)])


def test_decode_half_known_bit_patterns():
    # IEEE binary16: 0x3C00 = 1, 0xC000 = -2, 0x0001 = 2^-24, 0x7BFF = 65504
    # bfloat16: 0x3F80 = 1, 0xC040 = -3, 0x0001 = 2^-133
    f16 = np.array([0x3C00, 0xC000, 0x0001, 0x7BFF], np.uint16).reshape(1, 1, 2, 2)
    bf16 = np.array([0x3F80, 0xC040, 0x0001, 0x0000], np.uint16).reshape(1, 1, 2, 2)
    e = np.array([[3]], np.int8)
    got = oracle.decode_half(f16, e, "f16", 0)
    np.testing.assert_array_equal(got.ravel(), np.array([8 - 16j, 2.0 ** -21 + 65504 * 8j]))
    got = oracle.decode_half(bf16, np.array([[-2]], np.int8), "bf16", 0)
    np.testing.assert_array_equal(got.ravel(), np.array([0.25 - 0.75j, 2.0 ** -135]))


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_decode_half_line_axes(axis):
    nz, ny, nx = 3, 4, 5
    ones = np.full((nz, ny, nx, 2), 0x3C00, np.uint16)           # 1 + 1i everywhere
    shape = [(nz, ny), (nz, nx), (ny, nx)][axis]
    e = np.arange(np.prod(shape), dtype=np.int8).reshape(shape) - 5
    got = oracle.decode_half(ones, e, "f16", axis)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                ee = e[z, y] if axis == 0 else (e[z, x] if axis == 1 else e[y, x])
                assert got[z, y, x] == 2.0 ** ee * (1 + 1j)


def test_rel_l2_values():
    assert oracle.rel_l2([3 + 4j], [0]) == 5.0
    assert oracle.rel_l2([1 + 1j, 1], [1, 1]) == pytest.approx(1 / np.sqrt(2))
    assert oracle.rel_l2([2, 0], [2, 0]) == 0.0


# --------------------------------------------------------- real transforms
REAL_SHAPES = [(1, 1, 4), (3, 5, 8), (4, 6, 12), (2, 3, 16), (5, 4, 10)]


@pytest.mark.parametrize("nzyx", REAL_SHAPES, ids=str)
def test_rdft3d_matches_numpy_rfftn(nzyx):
    x = RNG.standard_normal(nzyx)
    assert oracle.rel_l2(oracle.rdft3d(x), np.fft.rfftn(x, axes=(0, 1, 2))) <= 1e-13


@pytest.mark.parametrize("nzyx", REAL_SHAPES, ids=str)
def test_irdft3d_matches_numpy_irfftn_on_any_half_spectrum(nzyx):
    # a half spectrum that is NOT the transform of a real grid: numpy's
    # irfftn also drops the imaginary parts of the kx = 0 and kx = nx/2 terms
    nz, ny, nx = nzyx
    h = RNG.standard_normal((nz, ny, nx // 2 + 1)) + 1j * RNG.standard_normal((nz, ny, nx // 2 + 1))
    ref = np.fft.irfftn(h, s=nzyx, axes=(0, 1, 2)) * (nx * ny * nz)
    assert oracle.rel_l2(oracle.irdft3d(h, nx), ref) <= 1e-13


@pytest.mark.parametrize("nzyx", REAL_SHAPES, ids=str)
def test_real_round_trip_is_n_identity(nzyx):
    x = RNG.standard_normal(nzyx)
    back = oracle.irdft3d(oracle.rdft3d(x), nzyx[2])
    assert oracle.rel_l2(back / x.size, x) <= 1e-13


def test_c2r_x_closed_forms():
    nx = 12
    n = np.arange(nx)
    g = np.zeros(nx // 2 + 1, complex)
    g[0] = 3 + 7j                      # imaginary part of the DC term drops out
    np.testing.assert_allclose(oracle.c2r_x(g, nx), np.full(nx, 3.0), atol=1e-14)
    g[:] = 0
    g[nx // 2] = -2 + 5j               # Nyquist term: alternating, imaginary part dropped
    np.testing.assert_allclose(oracle.c2r_x(g, nx), -2.0 * (-1.0) ** n, atol=1e-14)
    g[:] = 0
    c = 1.5 * np.exp(0.4j)
    g[2] = c                           # 2 |c| cos(2 pi 2 n / nx + arg c)
    np.testing.assert_allclose(oracle.c2r_x(g, nx), 3.0 * np.cos(2 * np.pi * 2 * n / nx + 0.4), atol=1e-13)


def test_rdft3d_of_cosine_gives_two_bins_in_the_half():
    nz, ny, nx = 3, 4, 16
    x = np.zeros((nz, ny, nx))
    x[:, :, :] = np.cos(2 * np.pi * 3 * np.arange(nx) / nx)
    r = oracle.rdft3d(x)
    ref = np.zeros((nz, ny, nx // 2 + 1), complex)
    ref[0, 0, 3] = nx * ny * nz / 2
    np.testing.assert_allclose(r, ref, atol=1e-11)


def test_real_exact_lines_match_full_transforms():
    nz, ny, nx = 6, 5, 20
    x = RNG.standard_normal((nz, ny, nx))
    r = oracle.rdft3d(x)
    kyz = [(0, 0), (4, 5), (2, 3)]
    assert oracle.rel_l2(oracle.rdft3d_lines(x, kyz), np.stack([r[kz, ky] for ky, kz in kyz])) <= 1e-13
    h = RNG.standard_normal(r.shape) + 1j * RNG.standard_normal(r.shape)
    b = oracle.irdft3d(h, nx)
    assert oracle.rel_l2(oracle.irdft3d_lines(h, nx, kyz), np.stack([b[z, y] for y, z in kyz])) <= 1e-13


def test_yz_sums_then_x_dft_is_the_exact_line():
    nz, ny, nx = 4, 3, 6
    x = rand_grid(nz, ny, nx)
    red = oracle.yz_sums(x, [(2, 1)], -1)
    full = oracle.dft3d_brute(x, -1)
    assert oracle.rel_l2(np.fft.fft(red[0]), full[1, 2]) <= 1e-13


# ------------------------------------------------------- PME convolution step
def _circular_convolution_brute(x, h):
    """(x (*) h)(n) = sum_j x(j) h(n - j mod shape), by direct loops."""
    nz, ny, nx = x.shape
    out = np.zeros_like(x)
    for z in range(nz):
        for y in range(ny):
            for xx in range(nx):
                acc = 0.0
                for jz in range(nz):
                    for jy in range(ny):
                        for jx in range(nx):
                            acc += x[jz, jy, jx] * h[(z - jz) % nz, (y - jy) % ny, (xx - jx) % nx]
                out[z, y, xx] = acc
    return out


def test_convolve_real_is_the_circular_convolution_theorem():
    # a real, even kernel h has a real spectrum; the step must give N (x (*) h)
    nz, ny, nx = 3, 4, 6
    x = RNG.standard_normal((nz, ny, nx))
    h = RNG.standard_normal((nz, ny, nx))
    h = (h + h[(-np.arange(nz)) % nz][:, (-np.arange(ny)) % ny][:, :, (-np.arange(nx)) % nx]) / 2
    g = np.fft.rfftn(h, axes=(0, 1, 2)).real          # the library FFT, not the oracle
    out, energy = oracle.convolve_real(x, g)
    conv = _circular_convolution_brute(x, h)
    assert oracle.rel_l2(out, x.size * conv) <= 1e-13
    # sum_k G |Q|^2 = N sum_j x(j) (x (*) h)(j)
    assert energy == pytest.approx(x.size * float(np.sum(x * conv)), rel=1e-12)


def test_convolve_real_unit_multiplier_is_n_identity_and_parseval():
    nz, ny, nx = 4, 5, 8
    x = RNG.standard_normal((nz, ny, nx))
    out, energy = oracle.convolve_real(x, np.ones((nz, ny, nx // 2 + 1)))
    assert oracle.rel_l2(out / x.size, x) <= 1e-13
    assert energy == pytest.approx(x.size * float(np.sum(x * x)), rel=1e-12)


def test_convolve_real_dc_only_multiplier():
    nz, ny, nx = 2, 3, 10
    x = RNG.standard_normal((nz, ny, nx))
    g = np.zeros((nz, ny, nx // 2 + 1))
    g[0, 0, 0] = 2.5
    out, energy = oracle.convolve_real(x, g)
    np.testing.assert_allclose(out, np.full(x.shape, 2.5 * x.sum()), atol=1e-12)
    assert energy == pytest.approx(2.5 * x.sum() ** 2, rel=1e-12)


def test_half_weights_count_every_full_bin_once():
    for nx in (4, 6, 16):
        assert oracle.half_weights(nx).sum() == nx


@pytest.mark.parametrize("nzyx", [(7, 11, 13), (2, 3, 97), (17, 1, 5)], ids=str)
def test_matches_numpy_on_lengths_with_large_prime_factors(nzyx):
    x = rand_grid(*nzyx)
    assert oracle.rel_l2(oracle.dft3d(x, -1), np.fft.fftn(x)) <= 1e-13
    assert oracle.rel_l2(oracle.dft3d(x, 1), np.fft.ifftn(x) * x.size) <= 1e-13
