"""GPU parity of the convolution plan (PME's reciprocal-space step: forward
real transform, product with a real multiplier, backward real transform, and
the energy sum) against the FP64 oracle, through the C ABI.

Small grids are compared element by element with ``oracle.convolve_real``.
At 512^3 the output is checked on sampled lines against the convolution
theorem with a separable 3-point stencil (whose multiplier is known in closed
form), and the fused plan is checked bit for bit against the same steps run
unfused (real forward plan, multiply, real backward plan).
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
REAL_NP = {C64: np.float32, C128: np.float64}
REAL_T = {C64: torch.float32, C128: torch.float64}
DT_IDS = {C64: "c64", C128: "c128"}

# (nx, ny, nz); (64, 48, 1) fuses along y, (16, 1, 8) has no y pass
SHAPES = [(8, 4, 2), (32, 20, 24), (64, 64, 64), (96, 30, 40), (128, 9, 16), (200, 12, 10), (64, 48, 1),
          (16, 1, 8), (256, 48, 36), (1024, 3, 4)]


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)
    sys.stdout.flush()


def run_conv(x, g, dtype, in_place=False, flags=0, energy=True):
    nz, ny, nx = x.shape
    d_x = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    d_g = torch.from_numpy(np.ascontiguousarray(g.astype(REAL_NP[dtype]))).cuda()
    d_out = d_x if in_place else torch.full_like(d_x, float("nan"))
    d_e = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda") if energy else None
    plan = croft.croft_plan_create_convolution(nx, ny, nz, dtype, flags)
    try:
        croft.croft_execute_convolution(plan, d_x, d_g, d_out, d_e)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(plan)
    return d_out.cpu().numpy(), (float(d_e.item()) if energy else None)


def multiplier(kind, dims, seed):
    nx, ny, nz = dims
    if kind == "pme":
        return synth.pme_influence(nx, ny, nz)
    return synth.normal_c((nz, ny, nx // 2 + 1), seed=seed).real


@pytest.mark.parametrize("kind", ["pme", "random"])
@pytest.mark.parametrize("dtype", [C64, C128], ids=DT_IDS.get)
@pytest.mark.parametrize("dims", SHAPES, ids=str)
def test_matches_oracle(dims, dtype, kind):
    nx, ny, nz = dims
    x = synth.normal_c((nz, ny, nx), seed=31).real.astype(REAL_NP[dtype])
    g = multiplier(kind, dims, 32)
    gs = g.astype(REAL_NP[dtype]).astype(np.float64)       # the multiplier as the GPU sees it
    got, energy = run_conv(x, g, dtype)
    ref, ref_e = oracle.convolve_real(x.astype(np.float64), gs)
    assert oracle.rel_l2(got, ref) <= TOL[dtype]
    # energy error relative to the sum of the magnitudes of its terms (a
    # multiplier of mixed sign may cancel)
    q = oracle.rdft3d(x.astype(np.float64))
    scale = float(np.sum(oracle.half_weights(nx) * np.abs(gs) * np.abs(q) ** 2))
    assert abs(energy - ref_e) <= TOL[dtype] * max(scale, 1e-300)


@pytest.mark.parametrize("dtype", [C64, C128], ids=DT_IDS.get)
def test_in_place_and_energy_are_reproducible(dtype):
    dims = (64, 40, 24)
    nx, ny, nz = dims
    x = synth.normal_c((nz, ny, nx), seed=33).real.astype(REAL_NP[dtype])
    g = synth.pme_influence(nx, ny, nz)
    a, ea = run_conv(x, g, dtype)
    b, eb = run_conv(x, g, dtype, in_place=True)
    c, ec = run_conv(x, g, dtype, energy=False)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(a, c)
    assert ea == eb and ec is None


@pytest.mark.parametrize("dtype", [C64, C128], ids=DT_IDS.get)
def test_measure_flag_gives_the_same_bits(dtype):
    dims = (128, 48, 32)
    nx, ny, nz = dims
    x = synth.normal_c((nz, ny, nx), seed=34).real.astype(REAL_NP[dtype])
    g = synth.pme_influence(nx, ny, nz)
    a, ea = run_conv(x, g, dtype)
    b, eb = run_conv(x, g, dtype, flags=croft.CROFT_MEASURE | croft.CROFT_NO_WISDOM)
    np.testing.assert_array_equal(a, b)
    assert ea == eb


def test_measure_from_a_wide_tile_start_stays_within_the_energy_partials(tmp_path, monkeypatch):
    """A fused length of 256 has two compiled candidates of different lines
    per tile (complex64: 16 and 32), so their block counts differ.  Seeded
    with the wider tile (fewer blocks), the plan's partials must still hold
    every block of the narrower one, which the autotuner launches; run twice,
    the second plan starting from the first one's recorded choice."""
    w = tmp_path / "w.txt"
    w.write_text("256 3 0 1 0\n")
    monkeypatch.setenv("CROFT_WISDOM", str(w))
    dims = (64, 32, 256)
    nx, ny, nz = dims
    x = synth.normal_c((nz, ny, nx), seed=35).real.astype(np.float32)
    g = synth.pme_influence(nx, ny, nz)
    ref, ref_e = oracle.convolve_real(x.astype(np.float64), g.astype(np.float32).astype(np.float64))
    outs = []
    for rep in range(2):
        got, energy = run_conv(x, g, C64, flags=croft.CROFT_MEASURE)
        assert oracle.rel_l2(got, ref) <= TOL[C64], rep
        assert abs(energy - ref_e) <= 1e-5 * abs(ref_e), rep
        outs.append((got, energy))
    plain, plain_e = run_conv(x, g, C64)
    for got, energy in outs:
        # the butterflies are the same in every candidate; the energy's
        # per-block partials follow the tile partition, so only its rounding
        # may differ
        np.testing.assert_array_equal(got, plain)
        assert abs(energy - plain_e) <= 1e-12 * abs(plain_e)


def unfused(d_x, d_g, dtype):
    """The same steps as separate plans: real forward, multiply, real backward."""
    nz, ny, nx = d_x.shape
    h = torch.empty((nz, ny, nx // 2 + 1), dtype=torch.complex64 if dtype == C64 else torch.complex128,
                    device="cuda")
    out = torch.empty_like(d_x)
    f = croft.croft_plan_create_real(nx, ny, nz, dtype, croft.CROFT_FORWARD, 0)
    b = croft.croft_plan_create_real(nx, ny, nz, dtype, croft.CROFT_BACKWARD, 0)
    try:
        croft.croft_execute(f, d_x, h)
        hr = torch.view_as_real(h)
        hr *= d_g[..., None]                      # (re g, im g), as the fused pass rounds it
        croft.croft_execute(b, h, out)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(f)
        croft.croft_plan_destroy(b)
    return out, h


@pytest.mark.parametrize("dtype", [C64, C128], ids=DT_IDS.get)
@pytest.mark.parametrize("dims", [(96, 30, 40), (256, 64, 48), (64, 48, 1)], ids=str)
def test_fused_equals_unfused_bitwise(dims, dtype):
    nx, ny, nz = dims
    x = synth.normal_c((nz, ny, nx), seed=35).real.astype(REAL_NP[dtype])
    g = synth.pme_influence(nx, ny, nz).astype(REAL_NP[dtype])
    d_x = torch.from_numpy(x).cuda()
    d_g = torch.from_numpy(g).cuda()
    ref, _ = unfused(d_x, d_g, dtype)
    got, _ = run_conv(x, g, dtype)
    np.testing.assert_array_equal(got, ref.cpu().numpy())


def test_bad_buffers_are_refused():
    nx, ny, nz = 32, 8, 8
    plan = croft.croft_plan_create_convolution(nx, ny, nz, C64, 0)
    try:
        info = croft.croft_plan_info(plan)
        assert info["convolution"] == 1 and info["real"] == 1
        assert [p["kind"] for p in info["passes"]] == [2, 1, 3, 1, 2]
        buf = torch.zeros(4 * nx * ny * nz, dtype=torch.float32, device="cuda")
        g = torch.zeros((nz, ny, nx // 2 + 1), dtype=torch.float32, device="cuda")
        with pytest.raises(ValueError, match="overlap"):
            croft.croft_execute_convolution(plan, buf, g, buf[nx:])
        with pytest.raises(ValueError, match="mul overlaps"):
            croft.croft_execute_convolution(plan, buf, buf[nx:], buf)
        with pytest.raises(ValueError, match="croft_execute_convolution"):
            croft.croft_execute(plan, buf, buf[2 * nx * ny * nz:])
    finally:
        croft.croft_plan_destroy(plan)
    real = croft.croft_plan_create_real(nx, ny, nz, C64, croft.CROFT_FORWARD, 0)
    try:
        with pytest.raises(ValueError, match="not a convolution plan"):
            croft.croft_execute_convolution(real, buf, g, buf[2 * nx * ny * nz:])
    finally:
        croft.croft_plan_destroy(real)


def stencil_multiplier(dims, coef):
    """G = prod_a (c0_a + 2 c1_a cos(2 pi k_a / n_a)): the spectrum of the real,
    even 3-point stencil h_a = (c1_a, c0_a, c1_a) in each axis."""
    nx, ny, nz = dims
    (ax, bx), (ay, by), (az, bz) = coef
    gx = ax + 2 * bx * np.cos(2 * np.pi * np.arange(nx // 2 + 1) / nx)
    gy = ay + 2 * by * np.cos(2 * np.pi * np.arange(ny) / ny)
    gz = az + 2 * bz * np.cos(2 * np.pi * np.arange(nz) / nz)
    return gz[:, None, None] * gy[None, :, None] * gx[None, None, :]


def stencil_line(x, y, z, coef):
    """(x (*) h)(:, y, z) for the separable 3-point stencil, in FP64."""
    nz, ny, nx = x.shape
    (ax, bx), (ay, by), (az, bz) = coef
    acc = np.zeros(nx)
    for dz, cz in ((-1, bz), (0, az), (1, bz)):
        for dy, cy in ((-1, by), (0, ay), (1, by)):
            row = x[(z + dz) % nz, (y + dy) % ny].astype(np.float64)
            acc += cz * cy * (ax * row + bx * (np.roll(row, 1) + np.roll(row, -1)))
    return acc


def test_pme_512_against_the_convolution_theorem():
    n = 512
    dims = (n, n, n)
    coef = ((0.5, 0.2), (0.6, -0.15), (0.4, 0.15))   # every factor stays positive
    log("PME 512^3 convolution: generate")
    grid, _ = synth.pme_grid(n, n, n, seed=3)
    x = grid.astype(np.float32)
    del grid
    g = stencil_multiplier(dims, coef).astype(np.float32)
    log("fused plan")
    got, energy = run_conv(x, g, C64)
    rng = np.random.Generator(np.random.PCG64(77))
    yz = [(0, 0), (n - 1, n - 1), (n // 2, n // 3)] + [tuple(int(v) for v in r) for r in rng.integers(0, n, (5, 2))]
    # the FP32 multiplier differs from the exact stencil spectrum by its rounding
    ref = np.stack([x.size * stencil_line(x, y, z, coef) for y, z in yz])
    got_l = np.stack([got[z, y] for y, z in yz])
    err = oracle.rel_l2(got_l, ref)
    log(f"lines rel-L2 {err:.3e}")
    assert err <= 1e-5
    log("energy: sum_k G |Q|^2 = N sum_j x (x (*) h)")
    conv_all = np.empty((n, n, n), np.float64)
    xd = x.astype(np.float64)
    (ax, bx), (ay, by), (az, bz) = coef
    t = ax * xd + bx * (np.roll(xd, 1, axis=2) + np.roll(xd, -1, axis=2))
    t = ay * t + by * (np.roll(t, 1, axis=1) + np.roll(t, -1, axis=1))
    conv_all[:] = az * t + bz * (np.roll(t, 1, axis=0) + np.roll(t, -1, axis=0))
    ref_e = x.size * float(np.sum(xd * conv_all))
    log(f"energy {energy:.9e} ref {ref_e:.9e}")
    assert abs(energy - ref_e) <= 1e-5 * abs(ref_e)


def test_pme_512_fused_equals_unfused_bitwise():
    n = 512
    grid, _ = synth.pme_grid(n, n, n, seed=3)
    x = grid.astype(np.float32)
    del grid
    g = synth.pme_influence(n, n, n).astype(np.float32)
    d_x = torch.from_numpy(x).cuda()
    d_g = torch.from_numpy(g).cuda()
    log("unfused")
    ref, h = unfused(d_x, d_g, C64)
    del h
    torch.cuda.empty_cache()
    log("fused")
    out = torch.empty_like(d_x)
    d_e = torch.zeros(1, dtype=torch.float64, device="cuda")
    plan = croft.croft_plan_create_convolution(n, n, n, C64, 0)
    try:
        croft.croft_execute_convolution(plan, d_x, d_g, out, d_e)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(plan)
    assert torch.equal(out, ref)
    log("done")
