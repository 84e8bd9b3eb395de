"""The strided candidates that fetch their next tile while the current one
finishes: into LDS (the first half, global_load_lds; persistent grids of
whole tiles, in 512- or 256-thread blocks) or, for 16-bit storage, into registers (with the input
exponents packed four to a register, loaded once per block where every
tile of the block shares them).  They run the same butterflies as the other
candidates of their length, so forcing one through the wisdom file must
give the default plan's bits; the grids are large enough that every block
runs several tiles (so the fetch of a next tile really happens), and the
first is also checked against exact oracle lines."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_04896_amd as croft
from paper_2002_04896_amd import synth
from gpu_helpers import HALF_TORCH, TOL

pytestmark = pytest.mark.gpu

C64, F16, BF16 = croft.CROFT_C64, croft.CROFT_C16F, croft.CROFT_C16B
FWD, BWD = croft.CROFT_FORWARD, croft.CROFT_BACKWARD

# (dtype, (nz, ny, nx), axis of the pass, length, candidates with the copy)
CASES = [
    (C64, (512, 256, 128), 2, 512, (17, 18, 19, 20)),
    (C64, (256, 512, 128), 1, 512, (17, 18, 19, 20)),
    (C64, (1024, 64, 256), 2, 1024, (10, 11, 12)),
    (F16, (512, 128, 256), 2, 512, (17, 18, 21, 22)),
    (BF16, (512, 128, 256), 2, 512, (17, 18, 21, 22)),
    (F16, (1024, 128, 128), 2, 1024, (10, 11)),
    # register prefetch: exponents once per block (z, nx = 256), once per
    # tile (z, nx = 100: the block's line stride is no multiple of nx; the
    # y pass: the exponents change with the plane), partial tiles (es = 2100)
    (F16, (512, 128, 256), 2, 512, (19, 20, 23, 24)),
    (BF16, (512, 128, 256), 2, 512, (19, 20, 23, 24)),
    (F16, (512, 64, 100), 2, 512, (19, 20, 23, 24)),
    (BF16, (512, 21, 100), 2, 512, (19, 20, 23, 24)),
    (F16, (128, 512, 256), 1, 512, (19, 20, 21, 22, 23, 24)),
]


def run(dtype, shape, direction, d_in, e_in):
    nz, ny, nx = shape
    plan = croft.croft_plan_create(nx, ny, nz, dtype, direction)
    try:
        out = torch.full_like(d_in, float("nan"))
        e_out = torch.full((ny, nx), 99, dtype=torch.int8, device="cuda")
        if dtype == C64:
            croft.croft_execute(plan, d_in, out)
        else:
            croft.croft_execute_scaled(plan, d_in, e_in, out, e_out)
        torch.cuda.synchronize()
        info = croft.croft_plan_info(plan)
    finally:
        croft.croft_plan_destroy(plan)
    return out, e_out, info


@pytest.mark.parametrize("case", range(len(CASES)))
def test_next_tile_fetch_candidates_give_identical_bits(case, tmp_path, monkeypatch):
    dtype, shape, axis, n, cands = CASES[case]
    nz, ny, nx = shape
    wisdom = tmp_path / "w.txt"
    monkeypatch.setenv("CROFT_WISDOM", str(wisdom))
    rng = np.random.Generator(np.random.PCG64(140 + case))
    if dtype == C64:
        x = (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(np.complex64)
        d_in = torch.from_numpy(x).cuda()
        e_in = None
    else:
        d_in = torch.from_numpy(rng.standard_normal(shape + (2,)).astype(np.float32)).cuda().to(HALF_TORCH[dtype])
        e_in = torch.from_numpy(rng.integers(-4, 5, size=(nz, ny)).astype(np.int8)).cuda()
    for direction in (FWD, BWD):
        wisdom.write_text(f"{n} 1 {dtype} 6 1 {axis}\n")      # a candidate without the copy
        ref, ref_e, _ = run(dtype, shape, direction, d_in, e_in)
        for cand in cands:
            for waves in (0, 1, 2):  # 0: one block per tile (a block copies its own tile's first half)
                print(f"dtype {dtype} shape {shape} axis {axis} cand {cand} waves {waves} dir {direction}",
                      flush=True)
                wisdom.write_text(f"{n} 1 {dtype} {cand} {waves} {axis}\n")
                got, got_e, info = run(dtype, shape, direction, d_in, e_in)
                assert info["passes"][axis]["blocks"] > 0
                bits = torch.int32 if dtype == C64 else torch.int16
                assert torch.equal(got.view(bits), ref.view(bits)), (cand, waves, direction)
                assert torch.equal(got_e, ref_e)
    if dtype == C64:
        kyz = [(0, 0), (ny - 1, nz - 1), (3, 7)]
        got = ref.cpu().numpy()       # the last direction (backward) of the reference
        lines = np.stack([got[kz, ky] for ky, kz in kyz])
        assert oracle.rel_l2(lines, oracle.dft3d_lines(x, kyz, BWD)) <= TOL[C64]


def test_half_tile_copy_falls_back_on_partial_tiles(tmp_path, monkeypatch):
    """es not a multiple of the tile's lines: the planner runs the twin
    (the dry-run test in test_abi_cpu.py checks which), and it is right."""
    wisdom = tmp_path / "w.txt"
    monkeypatch.setenv("CROFT_WISDOM", str(wisdom))
    wisdom.write_text("512 1 0 17 1 2\n")
    plan = croft.croft_plan_create(40, 21, 512, C64, FWD)        # es = 840: 27 tiles of 32, the last partial
    info = croft.croft_plan_info(plan)
    croft.croft_plan_destroy(plan)
    assert info["passes"][2]["lines_per_block"] == 32 and info["passes"][2]["blocks"] == 27
    x = synth.normal_c((512, 21, 40), seed=150)
    d = torch.from_numpy(x.astype(np.complex64)).cuda()
    out = torch.empty_like(d)
    plan = croft.croft_plan_create(40, 21, 512, C64, FWD)
    croft.croft_execute(plan, d, out)
    torch.cuda.synchronize()
    croft.croft_plan_destroy(plan)
    kyz = [(0, 0), (20, 511)]
    got = out.cpu().numpy()
    assert oracle.rel_l2(np.stack([got[kz, ky] for ky, kz in kyz]),
                         oracle.dft3d_lines(x.astype(np.complex64), kyz, FWD)) <= TOL[C64]
