"""GPU parity: the HIP path against the FP64 oracle on seeded inputs.

Sizes here are ones the oracle finishes in seconds; they span several blocks
and ragged tails, static and runtime-radix kernels, every dtype and both
directions.  Full-size configurations are in test_gpu_fullsize.py.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_04896_amd as croft
from paper_2002_04896_amd import synth
from gpu_helpers import HALF_KIND, TOL, run_fft, run_half, to_device

pytestmark = pytest.mark.gpu

C64, C128, F16, BF16 = croft.CROFT_C64, croft.CROFT_C128, croft.CROFT_C16F, croft.CROFT_C16B
FWD, BWD = croft.CROFT_FORWARD, croft.CROFT_BACKWARD


def test_config_32cube_c64_uniform_forward_and_roundtrip():
    # single forward 32^3 c64, Uniform[-1,1) re/im, seed 1; plus inverse round trip
    x = synth.uniform_c((32, 32, 32), seed=1)
    seen, y, _ = run_fft(x, C64, FWD)
    assert oracle.rel_l2(y, oracle.dft3d(seen, -1)) <= TOL[C64]
    d = to_device(y, C64)
    plan = croft.croft_plan_create(32, 32, 32, C64, BWD)
    back = torch.empty_like(d)
    croft.croft_execute(plan, d, back)
    torch.cuda.synchronize()
    croft.croft_plan_destroy(plan)
    assert oracle.rel_l2(back.cpu().numpy() / x.size, seen) <= 1e-5


def test_config_32cube_c128():
    x = synth.uniform_c((32, 32, 32), seed=1)
    seen, y, _ = run_fft(x, C128, FWD)
    assert oracle.rel_l2(y, oracle.dft3d(seen, -1)) <= TOL[C128]
    seen, y, _ = run_fft(x, C128, BWD)
    assert oracle.rel_l2(y, oracle.dft3d(seen, +1)) <= TOL[C128]


# (nz, ny, nx): non-cubic, ragged tiles, mixed radix, length-1 axes, runtime-radix lengths
SHAPES = [(100, 60, 48), (48, 100, 60), (27, 45, 60), (3, 128, 5), (8, 30, 1), (1, 1, 1),
          (1, 1, 8), (64, 1, 1), (80, 72, 96), (5, 3, 2), (16, 384, 12), (2, 6, 1000),
          (12, 3, 1024), (9, 2048, 2), (2, 2, 4096), (4096, 3, 2), (25, 36, 40),
          (1024, 3, 40), (5, 1024, 33),   # strided 1024: 32-line tiles with a ragged tail
          (4, 240, 120), (480, 2, 3), (3, 320, 192), (160, 5, 7),   # compiled 2^a 3^b 5^c lengths
          (3, 200, 288), (360, 3, 4), (2, 400, 3), (3, 2, 576), (640, 2, 3), (3, 720, 2), (2, 3, 768),
          (960, 2, 2)]


@pytest.mark.parametrize("shape", SHAPES, ids=str)
@pytest.mark.parametrize("dtype", [C64, C128], ids=["c64", "c128"])
@pytest.mark.parametrize("direction", [FWD, BWD], ids=["fwd", "bwd"])
def test_shapes_against_oracle(shape, dtype, direction):
    x = synth.normal_c(shape, seed=2)
    seen, y, after = run_fft(x, dtype, direction)
    assert oracle.rel_l2(y, oracle.dft3d(seen, direction)) <= TOL[dtype]
    assert np.array_equal(after, seen)                      # out of place keeps the input


def _random_shape(rng):
    # axis lengths: unit, small smooth, the batched lengths, powers of two up
    # to 1024, and primes (Bluestein); at most about 200 K elements
    pool = [1, 2, 3, 4, 5, 6, 8, 9, 12, 15, 16, 25, 27, 32, 48, 60, 64, 72, 80, 96, 100, 128, 256, 512, 1024,
            7, 11, 13, 17, 31, 37, 97]
    while True:
        shape = tuple(int(v) for v in rng.choice(pool, size=3))
        if np.prod(shape) <= 200_000:
            return shape


@pytest.mark.parametrize("case", range(24))
def test_random_shapes_against_oracle(case):
    rng = np.random.Generator(np.random.PCG64(1000 + case))
    shape = _random_shape(rng)
    dtype = (C64, C128)[int(rng.integers(2))]
    direction = (FWD, BWD)[int(rng.integers(2))]
    print(f"case {case}: shape {shape} dtype {dtype} dir {direction}", flush=True)
    x = synth.normal_c(shape, seed=case)
    seen, y, _ = run_fft(x, dtype, direction)
    assert oracle.rel_l2(y, oracle.dft3d(seen, direction)) <= TOL[dtype], (shape, dtype, direction)


@pytest.mark.parametrize("dtype", [C64, C128], ids=["c64", "c128"])
def test_in_place_equals_out_of_place_bitwise(dtype):
    x = synth.normal_c((40, 36, 50), seed=3)
    _, y_oop, _ = run_fft(x, dtype)
    _, y_ip, _ = run_fft(x, dtype, inplace=True)
    assert np.array_equal(y_oop, y_ip)


def test_repeat_runs_bitwise_identical():
    x = synth.normal_c((64, 48, 60), seed=4)
    runs = [run_fft(x, C64)[1] for _ in range(3)]
    assert np.array_equal(runs[0], runs[1]) and np.array_equal(runs[1], runs[2])


@pytest.mark.parametrize("dtype", [C64, C128], ids=["c64", "c128"])
def test_shifted_delta_closed_form(dtype):
    # delta at an asymmetric point of a non-cubic grid -> full plane wave
    nz, ny, nx = 20, 12, 30
    az, ay, ax = 3, 7, 11
    x = np.zeros((nz, ny, nx), complex)
    x[az, ay, ax] = 1
    _, y, _ = run_fft(x, dtype)
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    want = np.exp(-2j * np.pi * (kx * ax / nx + ky * ay / ny + kz * az / nz))
    assert oracle.rel_l2(y, want) <= TOL[dtype]


def test_constant_and_plane_wave_closed_forms():
    x = np.full((24, 20, 16), 0.5 - 0.25j)
    _, y, _ = run_fft(x, C64)
    want = np.zeros_like(x)
    want[0, 0, 0] = x.size * (0.5 - 0.25j)
    assert oracle.rel_l2(y, want) <= 1e-6
    jz, jy, jx = np.meshgrid(np.arange(24), np.arange(20), np.arange(16), indexing="ij")
    x = np.exp(2j * np.pi * (3 * jx / 16 + 5 * jy / 20 + 7 * jz / 24))
    _, y, _ = run_fft(x, C128)
    want = np.zeros_like(x)
    want[7, 5, 3] = x.size
    assert oracle.rel_l2(y, want) <= 1e-12


def test_generic_kernels_match_oracle_on_hot_lengths():
    # the runtime-radix kernels, forced, on lengths that normally run static kernels
    x = synth.normal_c((48, 60, 64), seed=5)
    seen, y, _ = run_fft(x, C64, flags=croft.CROFT_FORCE_GENERIC)
    assert oracle.rel_l2(y, oracle.dft3d(seen)) <= TOL[C64]
    seen, y, _ = run_fft(x, C128, BWD, flags=croft.CROFT_FORCE_GENERIC)
    assert oracle.rel_l2(y, oracle.dft3d(seen, +1)) <= TOL[C128]


@pytest.mark.parametrize("slabs", [2, 4, 8])
def test_slab_schedule_is_bitwise_equal_to_plain(slabs):
    x = synth.normal_c((64, 40, 48), seed=6)
    _, plain, _ = run_fft(x, C64)
    _, piped, _ = run_fft(x, C64, slabs=slabs)
    assert np.array_equal(plain, piped)


def check_half_output(out_bits, out_exp, kind):
    """Every z-line's largest |re|, |im| was scaled into [2^14, 2^15) before
    rounding (so it is in [2^14, 2^15] after), or the line is zero."""
    parts = out_bits.view(np.float16).astype(np.float64) if kind == "f16" else \
        (out_bits.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    peak = np.abs(parts).max(axis=(0, 3))                    # (ny, nx)
    ok = ((peak >= 2.0 ** 14) & (peak <= 2.0 ** 15)) | ((peak == 0) & (out_exp == 0))
    assert ok.all()


@pytest.mark.parametrize("dtype", [F16, BF16], ids=["f16", "bf16"])
# (512, 3, 40), (1024, 2, 36), (3, 1024, 40): one-line-per-lane strided passes
# (z at 512 and 1024, y at 1024) with ragged last tiles; (3, 640, 5),
# (768, 2, 3), (2, 720, 3): the XCD-ordered strided tiles of the larger
# compiled lengths
@pytest.mark.parametrize("shape", [(40, 48, 64), (27, 60, 45), (1, 16, 1), (6, 1, 100), (512, 3, 40),
                                   (1024, 2, 36), (3, 1024, 40), (3, 640, 5), (768, 2, 3), (2, 720, 3)],
                         ids=str)
def test_half_storage_against_oracle(dtype, shape):
    kind = HALF_KIND[dtype]
    v = synth.normal_c(shape, seed=7)
    data, e = synth.quantize_half(v, kind)
    exact_in = oracle.decode_half(data, e, kind, 0)
    for direction in (FWD, BWD):
        out, oe = run_half(data, e, dtype, direction)
        got = oracle.decode_half(out, oe, kind, 2)
        assert oracle.rel_l2(got, oracle.dft3d(exact_in, direction)) <= TOL[dtype]
        check_half_output(out, oe, kind)


@pytest.mark.parametrize("dtype", [F16, BF16], ids=["f16", "bf16"])
def test_half_in_place_slabs_and_null_exponents(dtype):
    kind = HALF_KIND[dtype]
    v = synth.normal_c((32, 24, 40), seed=8)
    data, e = synth.quantize_half(v, kind)
    ref_out, ref_e = run_half(data, e, dtype)
    out, oe = run_half(data, e, dtype, inplace=True)
    assert np.array_equal(out, ref_out) and np.array_equal(oe, ref_e)
    out, oe = run_half(data, e, dtype, slabs=4)
    assert np.array_equal(out, ref_out) and np.array_equal(oe, ref_e)
    out, oe = run_half(data, np.zeros_like(e), dtype, in_exp_null=True)
    got = oracle.decode_half(out, oe, kind, 2)
    assert oracle.rel_l2(got, oracle.dft3d(oracle.decode_half(data, np.zeros_like(e), kind, 0))) <= 5e-3


def test_half_all_zero_input():
    data = np.zeros((8, 8, 8, 2), np.uint16)
    out, oe = run_half(data, np.zeros((8, 8), np.int8), F16)
    assert not out.any() and not oe.any()


def test_batched_uneven_grids():
    dims = [(48, 60, 64), (128, 72, 80), (100, 96, 48), (60, 60, 60), (8, 1, 3), (45, 27, 2)]
    plan = croft.croft_plan_create_batched(dims, C64, FWD)
    offs = croft.croft_plan_batched_offsets(plan, len(dims))
    assert offs[0] == 0 and offs[-1] == sum(a * b * c for a, b, c in dims)
    xs = [synth.pme_grid(nx, ny, nz, seed=10 + i)[0].astype(complex) for i, (nx, ny, nz) in enumerate(dims)]
    flat = np.concatenate([x.ravel() for x in xs]).astype(np.complex64)
    d_in = torch.from_numpy(flat).cuda()
    d_out = torch.full_like(d_in, complex(float("nan"), 0))
    for _ in range(2):                      # second call replays the captured graph
        croft.croft_execute_batched(plan, d_in, d_out)
    torch.cuda.synchronize()
    croft.croft_plan_destroy(plan)
    out = d_out.cpu().numpy()
    for i, (nx, ny, nz) in enumerate(dims):
        seen = flat[offs[i]:offs[i + 1]].reshape(nz, ny, nx).astype(np.complex128)
        got = out[offs[i]:offs[i + 1]].reshape(nz, ny, nx)
        assert oracle.rel_l2(got, oracle.dft3d(seen)) <= TOL[C64], f"grid {i} {dims[i]}"


def test_profile_records_each_pass():
    plan = croft.croft_plan_create(64, 64, 64, C64, FWD)
    d = to_device(synth.normal_c((64, 64, 64), 9), C64)
    out = torch.empty_like(d)
    croft.croft_plan_profile(plan, True)
    for _ in range(3):
        croft.croft_execute(plan, d, out)
    ms, n = croft.croft_plan_profile_read(plan)
    croft.croft_plan_destroy(plan)
    assert n == 3 and all(m > 0 for m in ms[:3]) and ms[3] == 0


def test_execute_argument_errors_on_device():
    plan = croft.croft_plan_create(16, 16, 16, C64, FWD)
    d = torch.zeros((16, 16, 16), dtype=torch.complex64, device="cuda")
    big = torch.zeros((2 * 16 * 16 * 16,), dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError, match="overlap"):
        croft.croft_execute(plan, big, big[1:])
    with pytest.raises(ValueError, match="NULL"):
        croft.croft_execute(plan, 0, d)
    with pytest.raises(ValueError, match="scaled"):
        croft.croft_execute_scaled(plan, d, None, d, torch.zeros(256, dtype=torch.int8, device="cuda"))
    croft.croft_plan_destroy(plan)
    hplan = croft.croft_plan_create(16, 16, 16, F16, FWD)
    with pytest.raises(ValueError, match="half"):
        croft.croft_execute(hplan, d, d)
    with pytest.raises(ValueError, match="out_exp"):
        croft.croft_execute_scaled(hplan, d, None, d, None)
    croft.croft_plan_destroy(hplan)


@pytest.mark.parametrize("direction", [FWD, BWD], ids=["fwd", "bwd"])
@pytest.mark.parametrize("dtype", [C64, C128, F16], ids=["c64", "c128", "f16"])
@pytest.mark.parametrize("shape", [(6, 256, 512), (3, 1024, 20), (4, 512, 80), (2, 384, 96)], ids=str)
def test_every_compiled_candidate_gives_identical_bits(dtype, shape, direction, tmp_path, monkeypatch):
    """Every autotuner candidate (and persistent-grid size) runs the same
    arithmetic in the same order, so the outputs agree bit for bit, in both
    directions (each has its own instantiation); the default candidate is
    checked against the oracle elsewhere."""
    wisdom = tmp_path / "wisdom.txt"
    monkeypatch.setenv("CROFT_WISDOM", str(wisdom))
    nz, ny, nx = shape
    rng = np.random.Generator(np.random.PCG64(21))
    full = dtype in (C64, C128)
    if full:
        npdt = np.complex64 if dtype == C64 else np.complex128
        x = torch.from_numpy((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(npdt)).cuda()
        ein = None
    else:
        x = torch.from_numpy(rng.standard_normal(shape + (2,)).astype(np.float16)).cuda()
        ein = torch.zeros((nz, ny), dtype=torch.int8, device="cuda")

    def run():
        out = torch.full_like(x, float("nan"))
        eout = torch.full((ny, nx), 99, dtype=torch.int8, device="cuda")
        plan = croft.croft_plan_create(nx, ny, nz, dtype, direction)
        info = croft.croft_plan_info(plan)
        if full:
            croft.croft_execute(plan, x, out)
        else:
            croft.croft_execute_scaled(plan, x, ein, out, eout)
        torch.cuda.synchronize()
        croft.croft_plan_destroy(plan)
        return out.cpu(), eout.cpu(), info

    wisdom.write_text("")
    ref, ref_e, info = run()
    assert not torch.isnan(ref).any()
    lengths = {(p["n"], p["kind"]) for p in info["passes"]}
    tried = 0
    for n, kind in lengths:
        for cand in range(27):
            for waves in (0, 1, 3):
                wisdom.write_text(f"{n} {kind} {dtype} {cand} {waves}\n")
                got, got_e, ginfo = run()
                chosen = [p for p in ginfo["passes"] if (p["n"], p["kind"]) == (n, kind)]
                bits = {C64: torch.int32, C128: torch.int64}.get(dtype, torch.int16)
                assert torch.equal(got.view(bits), ref.view(bits)), \
                    (n, kind, cand, waves)
                assert torch.equal(got_e, ref_e)
                tried += 1
    assert tried >= 48


def test_measure_flag_autotunes_and_records_wisdom(tmp_path, monkeypatch):
    wisdom = tmp_path / "w.txt"
    monkeypatch.setenv("CROFT_WISDOM", str(wisdom))
    x = synth.normal_c((16, 64, 256), seed=22)
    seen, ref, _ = run_fft(x, C64)
    _, y, _ = run_fft(x, C64, flags=croft.CROFT_MEASURE)
    assert oracle.rel_l2(y, oracle.dft3d(seen)) <= TOL[C64]
    lines = [l.split() for l in wisdom.read_text().strip().split("\n")]
    # strided passes are recorded with their axis (y = 1, z = 2)
    assert {(int(l[0]), int(l[1]), int(l[5]) if len(l) == 6 else -1) for l in lines} == \
        {(256, 0, -1), (64, 1, 1), (16, 1, 2)}
    assert np.array_equal(y, ref)


@pytest.mark.parametrize("dtype,direction", [(C64, FWD), (C128, BWD)], ids=["c64-fwd", "c128-bwd"])
def test_batched_launch_forms_match_single_grid_plans_bitwise(dtype, direction):
    """The batched launch forms (one launch per pass, and one cooperative
    launch for every pass) run the same butterflies as the single-grid
    kernels: identical bits."""
    dims = [(48, 60, 64), (128, 72, 80), (100, 96, 48), (64, 64, 64), (80, 100, 72), (96, 128, 60),
            (8, 1, 3), (45, 27, 2), (1, 64, 1), (60, 1, 100), (128, 128, 48), (96, 72, 1)]
    rng = np.random.Generator(np.random.PCG64(31))
    total = sum(a * b * c for a, b, c in dims)
    npdt = np.complex64 if dtype == C64 else np.complex128
    flat = (rng.standard_normal(total) + 1j * rng.standard_normal(total)).astype(npdt)
    d_in = torch.from_numpy(flat).cuda()
    ref = torch.empty_like(d_in)
    offs = [0]
    for a, b, c in dims:
        offs.append(offs[-1] + a * b * c)
    for i, (nx, ny, nz) in enumerate(dims):
        p = croft.croft_plan_create(nx, ny, nz, dtype, direction)
        croft.croft_execute(p, d_in[offs[i]:offs[i + 1]], ref[offs[i]:offs[i + 1]])
        torch.cuda.synchronize()
        croft.croft_plan_destroy(p)
    for flags in (0, croft.CROFT_PERSISTENT, croft.CROFT_GRAPH,
                  croft.CROFT_PERSISTENT | croft.CROFT_GRAPH):
        plan = croft.croft_plan_create_batched(dims, dtype, direction, flags)
        for rep in range(3):                     # with CROFT_GRAPH: capture, then replays
            out = torch.full_like(d_in, complex(float("nan"), 0))
            croft.croft_execute_batched(plan, d_in, out)
            torch.cuda.synchronize()
            assert torch.equal(out.view(torch.float64 if dtype == C64 else torch.complex128),
                               ref.view(torch.float64 if dtype == C64 else torch.complex128)), (flags, rep)
        replay = croft.croft_plan_info(plan)["graph_replay"]
        croft.croft_plan_destroy(plan)
        assert replay == (1 if flags & croft.CROFT_GRAPH else 0), (flags, replay)
    seen = flat[offs[1]:offs[2]].reshape(80, 72, 128).astype(np.complex128)
    got = ref.cpu().numpy()[offs[1]:offs[2]].reshape(80, 72, 128)
    assert oracle.rel_l2(got, oracle.dft3d(seen, direction)) <= TOL[dtype]


@pytest.mark.parametrize("dims", [(64, 48, 60), (45, 27, 2)], ids=["batched-kernel", "own-launches"])
def test_batched_plan_of_one_grid_runs_it(dims):
    nx, ny, nz = dims
    rng = np.random.Generator(np.random.PCG64(32))
    x = (rng.standard_normal((nz, ny, nx)) + 1j * rng.standard_normal((nz, ny, nx))).astype(np.complex64)
    d_in = torch.from_numpy(x).cuda()
    ref = torch.empty_like(d_in)
    p = croft.croft_plan_create(nx, ny, nz, C64, FWD)
    croft.croft_execute(p, d_in, ref)
    croft.croft_plan_destroy(p)
    plan = croft.croft_plan_create_batched([dims], C64, FWD)
    try:
        with pytest.raises(ValueError, match="batched"):
            croft.croft_execute(plan, d_in, torch.empty_like(d_in))
        out = torch.full_like(d_in, complex(float("nan"), 0))
        croft.croft_execute_batched(plan, d_in, out)
        torch.cuda.synchronize()
        assert croft.croft_plan_info(plan)["batched_count"] == 1
    finally:
        croft.croft_plan_destroy(plan)
    assert torch.equal(out.view(torch.float64), ref.view(torch.float64))


def test_batched_in_place():
    dims = [(64, 48, 60), (72, 80, 96)]
    total = sum(a * b * c for a, b, c in dims)
    rng = np.random.Generator(np.random.PCG64(32))
    flat = (rng.standard_normal(total) + 1j * rng.standard_normal(total)).astype(np.complex64)
    outs = []
    for flags in (0, croft.CROFT_PERSISTENT, croft.CROFT_GRAPH):
        d = torch.from_numpy(flat).cuda()
        plan = croft.croft_plan_create_batched(dims, C64, FWD, flags)
        croft.croft_execute_batched(plan, d, d)
        torch.cuda.synchronize()
        croft.croft_plan_destroy(plan)
        outs.append(d.cpu().numpy())
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])
    seen = flat[:64 * 48 * 60].reshape(60, 48, 64).astype(np.complex128)
    assert oracle.rel_l2(outs[0][:64 * 48 * 60].reshape(60, 48, 64), oracle.dft3d(seen)) <= TOL[C64]


# ------------------------------------------------ slab schedule (paper Section 5.1, K)
# (nz, ny, nx): non-cubic grids whose slabs split z into 2, 4 and 8; ragged
# tiles along x and y, and runtime-radix passes (30 and 100)
SLAB_SHAPES = [(64, 40, 48), (16, 30, 100)]


@pytest.mark.parametrize("shape", SLAB_SHAPES, ids=str)
@pytest.mark.parametrize("slabs", [2, 4, 8])
@pytest.mark.parametrize("direction", [FWD, BWD], ids=["fwd", "bwd"])
def test_slab_schedule_against_oracle_c64(shape, slabs, direction):
    """K > 1 against the FP64 oracle, not only against the plain schedule."""
    x = synth.normal_c(shape, seed=60 + slabs)
    seen, y, after = run_fft(x, C64, direction, slabs=slabs)
    assert oracle.rel_l2(y, oracle.dft3d(seen, direction)) <= TOL[C64]
    assert np.array_equal(after, seen)
    _, plain, _ = run_fft(x, C64, direction)
    assert np.array_equal(y, plain)


@pytest.mark.parametrize("slabs", [2, 4, 8])
@pytest.mark.parametrize("direction", [FWD, BWD], ids=["fwd", "bwd"])
def test_slab_schedule_against_oracle_c128(slabs, direction):
    x = synth.normal_c((32, 24, 20), seed=70 + slabs)
    seen, y, _ = run_fft(x, C128, direction, slabs=slabs)
    assert oracle.rel_l2(y, oracle.dft3d(seen, direction)) <= TOL[C128]


@pytest.mark.parametrize("shape", SLAB_SHAPES, ids=str)
@pytest.mark.parametrize("slabs", [2, 4, 8])
@pytest.mark.parametrize("direction", [FWD, BWD], ids=["fwd", "bwd"])
@pytest.mark.parametrize("dtype", [F16, BF16], ids=["f16", "bf16"])
def test_slab_schedule_against_oracle_half(shape, slabs, direction, dtype):
    kind = HALF_KIND[dtype]
    v = synth.normal_c(shape, seed=80 + slabs)
    data, e = synth.quantize_half(v, kind)
    exact_in = oracle.decode_half(data, e, kind, 0)
    out, oe = run_half(data, e, dtype, direction, slabs=slabs)
    got = oracle.decode_half(out, oe, kind, 2)
    assert oracle.rel_l2(got, oracle.dft3d(exact_in, direction)) <= TOL[dtype]
    check_half_output(out, oe, kind)
    ref_out, ref_e = run_half(data, e, dtype, direction)
    assert np.array_equal(out, ref_out) and np.array_equal(oe, ref_e)


@pytest.mark.parametrize("dtype", [C64, F16], ids=["c64", "f16"])
def test_slab_count_zero_is_chosen_by_measurement_and_recorded(dtype, tmp_path, monkeypatch):
    """K = 0 with CROFT_MEASURE times K in {1, 2, 4, 8, 16} dividing nz and
    records the pick; a later K = 0 plan of the same grid and dtype without
    CROFT_MEASURE takes it; an explicit K is kept as given."""
    wisdom = tmp_path / "w.txt"
    monkeypatch.setenv("CROFT_WISDOM", str(wisdom))
    nz, ny, nx = 48, 40, 64
    plan = croft.croft_plan_create_ex(nx, ny, nz, dtype, FWD, croft.CROFT_MEASURE, 0)
    k = croft.croft_plan_info(plan)["slabs"]
    croft.croft_plan_destroy(plan)
    assert k in (1, 2, 4, 8, 16) and nz % k == 0
    recorded = [l.split() for l in wisdom.read_text().splitlines() if l.startswith("slabs")]
    assert recorded and recorded[-1] == ["slabs", str(nx), str(ny), str(nz), str(dtype), str(k)]
    # a recorded K is taken by a K = 0 plan; a K named in the file wins
    wisdom.write_text(wisdom.read_text() + f"slabs {nx} {ny} {nz} {dtype} 16\n")
    plan = croft.croft_plan_create_ex(nx, ny, nz, dtype, FWD, 0, 0)
    assert croft.croft_plan_info(plan)["slabs"] == 16
    croft.croft_plan_destroy(plan)
    plan = croft.croft_plan_create_ex(nx, ny, nz, dtype, FWD, 0, 4)
    assert croft.croft_plan_info(plan)["slabs"] == 4
    croft.croft_plan_destroy(plan)
    # with nothing recorded for a grid, K = 0 is the plain schedule
    plan = croft.croft_plan_create_ex(nx, ny, 7, dtype, FWD, 0, 0)
    assert croft.croft_plan_info(plan)["slabs"] == 1
    croft.croft_plan_destroy(plan)
    # the chosen K runs and matches the oracle
    if dtype == C64:
        x = synth.normal_c((nz, ny, nx), seed=90)
        seen, y, _ = run_fft(x, C64, FWD, slabs=0)
        assert oracle.rel_l2(y, oracle.dft3d(seen, FWD)) <= TOL[C64]


# ------------------------------------------ batched tile shapes (autotuned)
BATCH_LENGTHS = (48, 60, 64, 72, 80, 96, 100, 128)


@pytest.mark.parametrize("flags", [0, croft.CROFT_PERSISTENT], ids=["per-pass", "cooperative"])
def test_batched_tile_shapes_give_identical_bits(flags, tmp_path, monkeypatch):
    """Each batched length compiles two tile shapes (threads per line, lines
    per tile) for complex64; they run the same butterflies, so forcing the
    other shape for every (length, kind) through the wisdom file changes no
    bit, and CROFT_MEASURE records a choice per (length, kind) as kinds 4
    (contiguous) and 5 (strided)."""
    wisdom = tmp_path / "w.txt"
    monkeypatch.setenv("CROFT_WISDOM", str(wisdom))
    dims = [(48, 60, 64), (128, 72, 80), (100, 96, 48), (64, 64, 64), (80, 100, 72), (96, 128, 60)]
    rng = np.random.Generator(np.random.PCG64(33))
    total = sum(a * b * c for a, b, c in dims)
    flat = (rng.standard_normal(total) + 1j * rng.standard_normal(total)).astype(np.complex64)
    d_in = torch.from_numpy(flat).cuda()

    def run(fl):
        plan = croft.croft_plan_create_batched(dims, C64, FWD, fl)
        try:
            out = torch.full_like(d_in, complex(float("nan"), 0))
            croft.croft_execute_batched(plan, d_in, out)
            torch.cuda.synchronize()
        finally:
            croft.croft_plan_destroy(plan)
        return out

    wisdom.write_text("")
    ref = run(flags)
    wisdom.write_text("".join(f"{n} {4 + k} {C64} 1 0\n" for n in BATCH_LENGTHS for k in (0, 1)))
    other = run(flags)
    assert torch.equal(torch.view_as_real(other), torch.view_as_real(ref))
    wisdom.write_text("")
    tuned = run(flags | croft.CROFT_MEASURE)
    assert torch.equal(torch.view_as_real(tuned), torch.view_as_real(ref))
    rec = {(int(l.split()[0]), int(l.split()[1])) for l in wisdom.read_text().splitlines()
           if l.split()[1] in ("4", "5")}
    # x passes are contiguous (kind 4), y and z passes strided (kind 5)
    want = {(nx, 4) for nx, _, _ in dims} | {(n, 5) for _, ny, nz in dims for n in (ny, nz)}
    assert rec == want, rec
    offs = np.concatenate([[0], np.cumsum([a * b * c for a, b, c in dims])])
    got = other.cpu().numpy()
    for i, (nx, ny, nz) in enumerate(dims):
        seen = flat[offs[i]:offs[i + 1]].reshape(nz, ny, nx).astype(np.complex128)
        assert oracle.rel_l2(got[offs[i]:offs[i + 1]].reshape(nz, ny, nx), oracle.dft3d(seen)) <= TOL[C64], i
