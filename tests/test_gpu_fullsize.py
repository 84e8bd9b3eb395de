"""GPU parity at full workload sizes.

The oracle cannot transform these grids whole in seconds, so each test checks
exact output lines Y(., ky, kz) computed one by one by the oracle (O(N) per
line), plus properties that hold at any size: the round trip, the DC bin of a
charge grid (the total charge), Hermitian symmetry of a real input, and the
half-storage exponent rule.  Sizes and inputs are those of the benchmark
workloads: 256^3 and 384^3 normal, 512^3 and 1024^3 PME charge grids, 64
uneven PME grids, 512^3 half storage.
"""
import sys
import time

import numpy as np
import pytest
import torch

import oracle
import paper_2002_04896_amd as croft
from paper_2002_04896_amd import synth
from gpu_helpers import HALF_KIND, HALF_TORCH, TOL

pytestmark = pytest.mark.gpu

C64, F16, BF16 = croft.CROFT_C64, croft.CROFT_C16F, croft.CROFT_C16B
FWD, BWD = croft.CROFT_FORWARD, croft.CROFT_BACKWARD


def log(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)
    sys.stdout.flush()


def sample_kyz(ny, nz, count, seed):
    """(ky, kz) pairs: the corners plus seeded random ones."""
    rng = np.random.Generator(np.random.PCG64(seed))
    pts = [(0, 0), (ny - 1, nz - 1), (ny // 2, nz // 3)]
    pts += [(int(a), int(b)) for a, b in zip(rng.integers(0, ny, count), rng.integers(0, nz, count))]
    return pts


def execute(plan, d_in, d_out):
    croft.croft_execute(plan, d_in, d_out)
    torch.cuda.synchronize()


def lines_of(out_np, kyz):
    return np.stack([out_np[kz, ky, :] for ky, kz in kyz])


@pytest.mark.parametrize("n", [256, 384])
def test_normal_cubes_forward_inverse(n):
    log(f"normal {n}^3 c64: generate")
    x = synth.normal_c((n, n, n), seed=2).astype(np.complex64)
    d_in = torch.from_numpy(x).cuda()
    d_y = torch.empty_like(d_in)
    d_back = torch.empty_like(d_in)
    fwd = croft.croft_plan_create(n, n, n, C64, FWD)
    bwd = croft.croft_plan_create(n, n, n, C64, BWD)
    try:
        log("forward")
        execute(fwd, d_in, d_y)
        log("backward")
        execute(bwd, d_y, d_back)
    finally:
        croft.croft_plan_destroy(fwd)
        croft.croft_plan_destroy(bwd)
    seen = x.astype(np.complex128)
    kyz = sample_kyz(n, n, 5, seed=n)
    log("oracle lines (forward)")
    y = d_y.cpu().numpy()
    assert oracle.rel_l2(lines_of(y, kyz), oracle.dft3d_lines(seen, kyz, -1)) <= TOL[C64]
    log("oracle lines (inverse of the forward output)")
    yy = y.astype(np.complex128)
    back = d_back.cpu().numpy()
    assert oracle.rel_l2(lines_of(back, kyz), oracle.dft3d_lines(yy, kyz, +1)) <= TOL[C64]
    log("round trip")
    assert oracle.rel_l2(back / x.size, seen) <= 1e-5


@pytest.mark.parametrize("n", [512, 1024])
def test_pme_cubes(n):
    log(f"PME {n}^3 c64: generate")
    grid, qtot = synth.pme_grid(n, n, n, seed=3)
    x = grid.astype(np.complex64)
    del grid
    d_in = torch.from_numpy(x).cuda()
    d_out = torch.empty_like(d_in)
    plan = croft.croft_plan_create(n, n, n, C64, FWD)
    try:
        log("forward")
        execute(plan, d_in, d_out)
    finally:
        croft.croft_plan_destroy(plan)
    del d_in
    y = d_out.cpu().numpy()
    del d_out
    torch.cuda.empty_cache()
    # DC = sum of the FP32-rounded grid (= total charge up to the rounding of the input)
    log("DC and Hermitian symmetry")
    s = np.sum(x.real, dtype=np.float64)
    assert abs(y[0, 0, 0].real - s) <= 1e-5 * np.sqrt(np.sum(np.abs(y[0, 0, :]) ** 2))
    assert abs(s - qtot) <= 1e-3 * max(1.0, abs(qtot))
    rng = np.random.Generator(np.random.PCG64(n))
    k = rng.integers(0, n, size=(4096, 3))
    a = y[k[:, 2], k[:, 1], k[:, 0]]
    b = y[(-k[:, 2]) % n, (-k[:, 1]) % n, (-k[:, 0]) % n]
    assert oracle.rel_l2(a, np.conj(b)) <= 1e-5
    log("oracle lines")
    kyz = sample_kyz(n, n, 5, seed=n + 1)   # 8 exact lines
    ref = oracle.dft3d_lines(x, kyz, -1)
    assert oracle.rel_l2(lines_of(y, kyz), ref) <= TOL[C64]
    log("done")


def test_batched_64_uneven_pme_grids():
    dims = [tuple(int(v) for v in d) for d in synth.batch_dims(4)]
    log(f"batch of {len(dims)} grids: generate")
    grids = [synth.pme_grid(nx, ny, nz, seed=400 + i)[0] for i, (nx, ny, nz) in enumerate(dims)]
    flat = np.concatenate([g.ravel() for g in grids]).astype(np.complex64)
    plan = croft.croft_plan_create_batched(dims, C64, FWD)
    offs = croft.croft_plan_batched_offsets(plan, len(dims))
    d_in = torch.from_numpy(flat).cuda()
    d_out = torch.full_like(d_in, complex(float("nan"), 0))
    try:
        croft.croft_execute_batched(plan, d_in, d_out)
        croft.croft_execute_batched(plan, d_in, d_out)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(plan)
    out = d_out.cpu().numpy()
    log("oracle lines per grid")
    errs = []
    for i, (nx, ny, nz) in enumerate(dims):
        seen = flat[offs[i]:offs[i + 1]].reshape(nz, ny, nx).astype(np.complex128)
        got = out[offs[i]:offs[i + 1]].reshape(nz, ny, nx)
        kyz = sample_kyz(ny, nz, 2, seed=i)
        errs.append(oracle.rel_l2(lines_of(got, kyz), oracle.dft3d_lines(seen, kyz, -1)))
        assert abs(got[0, 0, 0].real - seen.real.sum()) <= 1e-4 * max(1.0, np.abs(got[0, 0, :]).max())
    assert max(errs) <= TOL[C64], errs


@pytest.mark.parametrize("dtype", [F16, BF16], ids=["f16", "bf16"])
def test_half_storage_512(dtype):
    n = 512
    kind = HALF_KIND[dtype]
    log(f"half {kind} 512^3: generate")
    v = synth.normal_c((n, n, n), seed=5)
    data, e = synth.quantize_half(v, kind)
    d_in = torch.from_numpy(data.view(np.int16)).cuda().view(HALF_TORCH[dtype])
    d_out = torch.empty_like(d_in)
    e_in = torch.from_numpy(e).cuda()
    e_out = torch.full((n, n), 99, dtype=torch.int8, device="cuda")
    plan = croft.croft_plan_create(n, n, n, dtype, FWD)
    try:
        croft.croft_execute_scaled(plan, d_in, e_in, d_out, e_out)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(plan)
    out = d_out.view(torch.int16).cpu().numpy().view(np.uint16)
    oe = e_out.cpu().numpy()
    log("exponent rule")
    parts = out.view(np.float16).astype(np.float32) if kind == "f16" else \
        (out.astype(np.uint32) << 16).view(np.float32)
    peak = np.abs(parts).max(axis=(0, 3))
    assert np.all((peak >= 2.0 ** 14) & (peak <= 2.0 ** 15))
    log("oracle lines of the decoded input")
    exact_in = oracle.decode_half(data, e, kind, 0)
    kyz = sample_kyz(n, n, 5, seed=7)
    # sampled line i holds z-lines (x, ky_i): its exponents are oe[ky_i, :]
    got = oracle.decode_half(np.stack([out[kz, ky] for ky, kz in kyz])[:, None],
                             np.stack([oe[ky] for ky, kz in kyz]), kind, 1)[:, 0]
    ref = oracle.dft3d_lines(exact_in, kyz, -1)
    err = oracle.rel_l2(got, ref)
    log(f"{kind} rel-L2 vs oracle of the stored input: {err:.3e}")
    assert err <= TOL[dtype]
    # for information: against the oracle of the input before quantisation
    # (adds the input's own 16-bit rounding)
    err_orig = oracle.rel_l2(got, oracle.dft3d_lines(v, kyz, -1))
    log(f"{kind} rel-L2 vs oracle of the unquantised input: {err_orig:.3e}")
    assert err_orig <= 2 * TOL[dtype]
