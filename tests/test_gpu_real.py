"""GPU parity of the real transforms -- real grid to half spectrum (forward)
and half spectrum to real grid (backward) -- against the FP64 oracle, through
the C ABI.  Shapes span several tiles of the real x pass with ragged tails,
every compiled half length class (powers of two up to 4096 and the 3/5-smooth
ones), unit y or z axes, and the 512^3 PME charge grid on sampled exact lines.
"""
import sys
import time

import numpy as np
import pytest
import torch

import oracle
import paper_2002_04896_amd as croft
from paper_2002_04896_amd import synth
from gpu_helpers import TOL

pytestmark = pytest.mark.gpu

C64, C128 = croft.CROFT_C64, croft.CROFT_C128
FWD, BWD = croft.CROFT_FORWARD, croft.CROFT_BACKWARD
REAL_NP = {C64: np.float32, C128: np.float64}
CPLX_NP = {C64: np.complex64, C128: np.complex128}
DT_IDS = {C64: "c64", C128: "c128"}

# (nx, ny, nz): nx/2 = 2, 4, 8, 16, 32, 48, 100, 64, 384, 128, 512, 4096
SHAPES = [(4, 1, 1), (8, 4, 2), (16, 1, 8), (32, 20, 24), (64, 64, 64), (96, 30, 40), (200, 12, 10),
          (128, 9, 15), (768, 6, 5), (256, 48, 36), (1024, 3, 5), (8192, 2, 3)]


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)
    sys.stdout.flush()


def run_real(arr, dims, dtype, direction, flags=0):
    """One real transform of numpy array `arr` on the GPU: (output, input after the call)."""
    nx, ny, nz = dims
    d_in = torch.from_numpy(np.ascontiguousarray(arr)).cuda()
    if direction == FWD:
        d_out = torch.full((nz, ny, nx // 2 + 1), complex(float("nan"), float("nan")),
                           dtype=torch.complex64 if dtype == C64 else torch.complex128, device="cuda")
    else:
        d_out = torch.full((nz, ny, nx), float("nan"),
                           dtype=torch.float32 if dtype == C64 else torch.float64, device="cuda")
    plan = croft.croft_plan_create_real(nx, ny, nz, dtype, direction, flags)
    try:
        croft.croft_execute(plan, d_in, d_out)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(plan)
    return d_out.cpu().numpy(), d_in.cpu().numpy()


def real_grid(dims, seed, dtype):
    nx, ny, nz = dims
    return synth.normal_c((nz, ny, nx), seed=seed).real.astype(REAL_NP[dtype])


def half_spectrum(dims, seed, dtype):
    """Any half spectrum (not the transform of a real grid): the imaginary parts
    of its kx = 0 and kx = nx/2 terms must drop out of the backward result."""
    nx, ny, nz = dims
    return synth.normal_c((nz, ny, nx // 2 + 1), seed=seed).astype(CPLX_NP[dtype])


@pytest.mark.parametrize("dtype", [C64, C128], ids=DT_IDS.get)
@pytest.mark.parametrize("dims", SHAPES, ids=str)
def test_forward_matches_oracle(dims, dtype):
    x = real_grid(dims, 11, dtype)
    got, after = run_real(x, dims, dtype, FWD)
    np.testing.assert_array_equal(after, x)
    assert got.shape == (dims[2], dims[1], dims[0] // 2 + 1)
    assert oracle.rel_l2(got, oracle.rdft3d(x.astype(np.float64))) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [C64, C128], ids=DT_IDS.get)
@pytest.mark.parametrize("dims", SHAPES, ids=str)
def test_backward_matches_oracle(dims, dtype):
    h = half_spectrum(dims, 12, dtype)
    got, after = run_real(h, dims, dtype, BWD)
    np.testing.assert_array_equal(after, h)
    assert got.shape == (dims[2], dims[1], dims[0])
    assert oracle.rel_l2(got, oracle.irdft3d(h.astype(np.complex128), dims[0])) <= TOL[dtype]


@pytest.mark.parametrize("dtype", [C64, C128], ids=DT_IDS.get)
def test_round_trip_of_pme_grid(dtype):
    dims = (64, 48, 40)
    grid, _ = synth.pme_grid(dims[0], dims[1], dims[2], seed=21)
    x = grid.real.astype(REAL_NP[dtype])
    h, _ = run_real(x, dims, dtype, FWD)
    back, _ = run_real(h, dims, dtype, BWD)
    assert oracle.rel_l2(back / x.size, x) <= 10 * TOL[dtype]
    # the spectrum of a real grid: DC is the total, kx = 0 and nx/2 planes Hermitian in (ky, kz)
    assert abs(h[0, 0, 0].real - x.astype(np.float64).sum()) <= 1e-5 * np.abs(h[0, 0]).max() + 1e-12
    for kx in (0, dims[0] // 2):
        plane = h[:, :, kx]
        mirror = np.conj(np.roll(plane[::-1, ::-1], 1, axis=(0, 1)))
        assert oracle.rel_l2(plane, mirror) <= TOL[dtype]


def test_forward_equals_first_half_of_complex_transform():
    dims = (128, 24, 20)
    x = real_grid(dims, 13, C128)
    got, _ = run_real(x, dims, C128, FWD)
    nx, ny, nz = dims
    d = torch.from_numpy(x.astype(np.complex128)).cuda()
    out = torch.empty_like(d)
    plan = croft.croft_plan_create(nx, ny, nz, C128, FWD)
    try:
        croft.croft_execute(plan, d, out)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(plan)
    assert oracle.rel_l2(got, out.cpu().numpy()[:, :, : nx // 2 + 1]) <= 1e-13


@pytest.mark.parametrize("direction", [FWD, BWD], ids=["fwd", "bwd"])
def test_measure_flag_gives_the_same_bits(direction):
    dims = (256, 40, 24)
    a = real_grid(dims, 14, C64) if direction == FWD else half_spectrum(dims, 14, C64)
    ref, _ = run_real(a, dims, C64, direction)
    got, _ = run_real(a, dims, C64, direction, croft.CROFT_MEASURE | croft.CROFT_NO_WISDOM)
    np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))


def test_real_plan_info_and_buffer_rules():
    nx, ny, nz = 64, 16, 8
    f = croft.croft_plan_create_real(nx, ny, nz, C64, FWD, 0)
    b = croft.croft_plan_create_real(nx, ny, nz, C64, BWD, 0)
    try:
        fi, bi = croft.croft_plan_info(f), croft.croft_plan_info(b)
        assert fi["real"] == 1 and bi["real"] == 1
        assert [p["kind"] for p in fi["passes"]] == [2, 1, 1]
        assert [p["axis"] for p in bi["passes"]] == [2, 1, 0]
        spec = (nx // 2 + 1) * ny * nz * 8
        assert bi["work_bytes"] >= spec > fi["work_bytes"]
        assert fi["algorithmic_bytes"] == nx * ny * nz * 4 + spec + 4 * spec
        x = torch.zeros(nz * ny * nx * 4, dtype=torch.float32, device="cuda")
        with pytest.raises(ValueError, match="out of place"):
            croft.croft_execute(f, x, x)
        with pytest.raises(ValueError, match="out of place"):
            croft.croft_execute(f, x, x[nx * ny * nz // 2:])  # spectrum overlaps the real grid
        with pytest.raises(ValueError, match="batched"):
            croft.croft_execute_batched(f, x, x[2 * nx * ny * nz:])
    finally:
        croft.croft_plan_destroy(f)
        croft.croft_plan_destroy(b)


def test_pme_512_forward_and_backward_lines():
    n = 512
    dims = (n, n, n)
    log("PME 512^3 real: generate")
    grid, qtot = synth.pme_grid(n, n, n, seed=3)
    x = grid.real.astype(np.float32)
    del grid
    d_x = torch.from_numpy(x).cuda()
    d_h = torch.empty((n, n, n // 2 + 1), dtype=torch.complex64, device="cuda")
    d_back = torch.empty_like(d_x)
    fwd = croft.croft_plan_create_real(n, n, n, C64, FWD, 0)
    bwd = croft.croft_plan_create_real(n, n, n, C64, BWD, 0)
    try:
        log("forward")
        croft.croft_execute(fwd, d_x, d_h)
        log("backward")
        croft.croft_execute(bwd, d_h, d_back)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(fwd)
        croft.croft_plan_destroy(bwd)
    h = d_h.cpu().numpy()
    back = d_back.cpu().numpy()
    del d_x, d_h, d_back
    torch.cuda.empty_cache()
    log("DC and round trip")
    s = np.sum(x, dtype=np.float64)
    assert abs(h[0, 0, 0].real - s) <= 1e-5 * np.sqrt(np.sum(np.abs(h[0, 0, :]) ** 2))
    assert abs(s - qtot) <= 1e-3 * max(1.0, abs(qtot))
    assert oracle.rel_l2(back / x.size, x) <= 1e-5
    rng = np.random.Generator(np.random.PCG64(512))
    kyz = [(0, 0), (n - 1, n - 1), (n // 2, n // 3)] + [tuple(int(v) for v in r) for r in rng.integers(0, n, (3, 2))]
    log("oracle forward lines")
    got = np.stack([h[kz, ky] for ky, kz in kyz])
    assert oracle.rel_l2(got, oracle.rdft3d_lines(x, kyz)) <= TOL[C64]
    log("oracle backward lines")
    got = np.stack([back[z, y] for y, z in kyz])
    assert oracle.rel_l2(got, oracle.irdft3d_lines(h, n, kyz)) <= TOL[C64]
    log("done")


def test_python_wrappers_check_shapes_and_run():
    nx, ny, nz = 32, 12, 10
    x = torch.from_numpy(real_grid((nx, ny, nz), 15, C64)).cuda()
    h = torch.empty((nz, ny, nx // 2 + 1), dtype=torch.complex64, device="cuda")
    back = torch.empty_like(x)
    f = croft.RealPlan(nx, ny, nz, C64, FWD)
    b = croft.RealPlan(nx, ny, nz, C64, BWD)
    f(x, h)
    b(h, back)
    torch.cuda.synchronize()
    assert oracle.rel_l2(back.cpu().numpy() / x.numel(), x.cpu().numpy()) <= 10 * TOL[C64]
    with pytest.raises(ValueError, match="shape"):
        f(x, torch.empty((nz, ny, nx), dtype=torch.complex64, device="cuda"))
    with pytest.raises(ValueError, match="dtype"):
        b(h, torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda"))
    g = torch.ones((nz, ny, nx // 2 + 1), dtype=torch.float32, device="cuda")
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    conv = croft.ConvolutionPlan(nx, ny, nz, C64)
    out = conv(x, g, torch.empty_like(x), e)
    torch.cuda.synchronize()
    xs = x.cpu().numpy().astype(np.float64)
    assert oracle.rel_l2(out.cpu().numpy() / x.numel(), xs) <= 10 * TOL[C64]
    assert abs(e.item() - x.numel() * float(np.sum(xs * xs))) <= 1e-5 * x.numel() * float(np.sum(xs * xs))
    with pytest.raises(ValueError, match="mul"):
        conv(x, torch.ones((nz, ny, nx), dtype=torch.float32, device="cuda"), torch.empty_like(x))
    for p in (f, b, conv):
        p.destroy()
