"""The unfused schedule (CROFT_UNFUSED): the paper's Option 2 (Section 5.1),
the three axis FFTs on contiguous lines with standalone LDS-tiled transposes
of the whole grid between them, kept as the measured baseline of the fused
passes.  Checked against the FP64 oracle and, bit for bit, against the fused
plan (the same butterflies in the same order: only the data movement
differs)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_04896_amd as croft
from paper_2002_04896_amd import synth
from gpu_helpers import TOL, run_fft

pytestmark = pytest.mark.gpu

C64, C128 = croft.CROFT_C64, croft.CROFT_C128
FWD, BWD = croft.CROFT_FORWARD, croft.CROFT_BACKWARD

# (nz, ny, nx): tile edges (64) crossed with ragged remainders, unit axes,
# mixed radix, runtime-radix and Bluestein lengths
SHAPES = [(40, 48, 64), (100, 60, 48), (3, 130, 70), (1, 1, 96), (64, 1, 1), (5, 1, 200), (17, 19, 23),
          (128, 128, 2), (2, 1000, 3)]


@pytest.mark.parametrize("shape", SHAPES, ids=str)
@pytest.mark.parametrize("dtype", [C64, C128], ids=["c64", "c128"])
@pytest.mark.parametrize("direction", [FWD, BWD], ids=["fwd", "bwd"])
def test_unfused_against_oracle_and_fused(shape, dtype, direction):
    x = synth.normal_c(shape, seed=120)
    seen, y, after = run_fft(x, dtype, direction, flags=croft.CROFT_UNFUSED)
    assert oracle.rel_l2(y, oracle.dft3d(seen, direction)) <= TOL[dtype]
    assert np.array_equal(after, seen)
    _, fused, _ = run_fft(x, dtype, direction)
    assert np.array_equal(y, fused)


def test_unfused_in_place_and_profiled_launches():
    nz, ny, nx = 24, 40, 72
    x = synth.normal_c((nz, ny, nx), seed=121)
    _, ref, _ = run_fft(x, C64, FWD, flags=croft.CROFT_UNFUSED)
    _, got, _ = run_fft(x, C64, FWD, flags=croft.CROFT_UNFUSED, inplace=True)
    assert np.array_equal(got, ref)
    plan = croft.croft_plan_create_ex(nx, ny, nz, C64, FWD, croft.CROFT_UNFUSED, 0)
    d = torch.from_numpy(x.astype(np.complex64)).cuda()
    out = torch.empty_like(d)
    croft.croft_plan_profile(plan, True)
    croft.croft_execute(plan, d, out)
    ms, n = croft.croft_plan_profile_read(plan)
    info = croft.croft_plan_info(plan)
    croft.croft_plan_destroy(plan)
    assert n == 1 and all(m > 0 for m in ms[:6]) and ms[6] == 0   # three FFTs, three transposes
    assert info["work_bytes"] >= nx * ny * nz * 8                 # the work grid
