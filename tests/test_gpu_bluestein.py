"""GPU parity of lengths with prime factors above 5 (Bluestein's algorithm),
against the FP64 oracle (a naive DFT, valid for every length), through the
C ABI: on the contiguous and the strided axes, forward and backward, every
dtype, inside real plans and as the loose grids of batched plans."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_04896_amd as croft
from paper_2002_04896_amd import synth
from gpu_helpers import HALF_KIND, TOL, run_fft, run_half

pytestmark = pytest.mark.gpu

C64, C128, F16, BF16 = croft.CROFT_C64, croft.CROFT_C128, croft.CROFT_C16F, croft.CROFT_C16B
FWD, BWD = croft.CROFT_FORWARD, croft.CROFT_BACKWARD

# (nx, ny, nz): primes on x (contiguous), on y and z (strided), a long prime,
# and prime lengths mixed with the compiled ones; together they use every
# convolution length the kernel is compiled for up to 4096 (16 .. 4096:
# 7, 11, 17, 41, 97, 131, 509, 1009, 2039)
SHAPES = [(7, 11, 13), (97, 9, 5), (1009, 3, 2), (17, 256, 19), (128, 131, 2), (60, 7, 64), (2039, 3, 2),
          (41, 37, 43), (509, 4, 3), (6, 509, 2)]


@pytest.mark.parametrize("direction", [FWD, BWD], ids=["fwd", "bwd"])
@pytest.mark.parametrize("dtype", [C64, C128], ids=["c64", "c128"])
@pytest.mark.parametrize("dims", SHAPES, ids=str)
def test_matches_oracle(dims, dtype, direction):
    nx, ny, nz = dims
    x = synth.normal_c((nz, ny, nx), seed=41)
    seen, got, after = run_fft(x, dtype, direction)
    assert oracle.rel_l2(got, oracle.dft3d(seen, direction)) <= TOL[dtype]
    np.testing.assert_array_equal(after, seen)


def test_longest_prime_complex64():
    x = synth.normal_c((1, 2, 4093), seed=42)
    seen, got, _ = run_fft(x, C64, FWD)
    assert oracle.rel_l2(got, oracle.dft3d(seen, FWD)) <= TOL[C64]


@pytest.mark.parametrize("dtype", [C64, C128], ids=["c64", "c128"])
def test_round_trip_and_in_place(dtype):
    nx, ny, nz = 23, 29, 31
    x = synth.normal_c((nz, ny, nx), seed=43)
    seen, y, _ = run_fft(x, dtype, FWD)
    _, y2, _ = run_fft(x, dtype, FWD, inplace=True)
    np.testing.assert_array_equal(y, y2)
    _, back, _ = run_fft(y, dtype, BWD)
    assert oracle.rel_l2(back / x.size, seen) <= 10 * TOL[dtype]


@pytest.mark.parametrize("dtype", [F16, BF16], ids=["f16", "bf16"])
def test_half_storage(dtype):
    nx, ny, nz = 13, 40, 11
    kind = HALF_KIND[dtype]
    data, e = synth.quantize_half(synth.normal_c((nz, ny, nx), seed=44), kind)
    out, oe = run_half(data, e, dtype)
    exact_in = oracle.decode_half(data, e, kind, 0)
    got = oracle.decode_half(out, oe, kind, 2)
    assert oracle.rel_l2(got, oracle.dft3d(exact_in, FWD)) <= TOL[dtype]


def test_real_plan_with_prime_y_and_z():
    nx, ny, nz = 64, 7, 11
    x = synth.normal_c((nz, ny, nx), seed=45).real.astype(np.float32)
    d = torch.from_numpy(x).cuda()
    h = torch.empty((nz, ny, nx // 2 + 1), dtype=torch.complex64, device="cuda")
    back = torch.empty_like(d)
    f = croft.croft_plan_create_real(nx, ny, nz, C64, FWD, 0)
    b = croft.croft_plan_create_real(nx, ny, nz, C64, BWD, 0)
    try:
        croft.croft_execute(f, d, h)
        croft.croft_execute(b, h, back)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(f)
        croft.croft_plan_destroy(b)
    assert oracle.rel_l2(h.cpu().numpy(), oracle.rdft3d(x.astype(np.float64))) <= TOL[C64]
    assert oracle.rel_l2(back.cpu().numpy() / x.size, x) <= 10 * TOL[C64]


def test_batched_plan_runs_prime_grids_with_their_own_launches():
    dims = [(48, 60, 64), (7, 8, 9), (64, 64, 64), (11, 13, 2)]
    total = sum(a * b * c for a, b, c in dims)
    flat = synth.normal_c((total,), seed=46).astype(np.complex64)
    d_in = torch.from_numpy(flat).cuda()
    out = torch.full_like(d_in, complex(float("nan"), 0))
    plan = croft.croft_plan_create_batched(dims, C64, FWD)
    try:
        offs = croft.croft_plan_batched_offsets(plan, len(dims))
        croft.croft_execute_batched(plan, d_in, out)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(plan)
    got = out.cpu().numpy()
    for i, (nx, ny, nz) in enumerate(dims):
        seen = flat[offs[i]:offs[i + 1]].reshape(nz, ny, nx).astype(np.complex128)
        ref = oracle.dft3d(seen, FWD)
        assert oracle.rel_l2(got[offs[i]:offs[i + 1]].reshape(nz, ny, nx), ref) <= TOL[C64], (i, dims[i])
