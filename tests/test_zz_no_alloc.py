"""The allocation-free half-storage execute (croft_execute_scaled_noalloc)
against croft_execute_scaled, through the C ABI.

Both run the same kernels; the allocation-free call keeps the intermediate
per-line exponents in the GPU's static scratch array instead of the plan's
own.  Its output and exponents must equal the plan's execute bit for bit, on
consecutive calls that share that array, the second on a smaller grid.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2002_04896_amd as croft
from paper_2002_04896_amd import synth
from gpu_helpers import HALF_KIND, HALF_TORCH, TOL

pytestmark = pytest.mark.gpu

F16, BF16 = croft.CROFT_C16F, croft.CROFT_C16B
FWD, BWD = croft.CROFT_FORWARD, croft.CROFT_BACKWARD


def _inputs(shape, dtype, seed):
    kind = HALF_KIND[dtype]
    v = synth.normal_c(shape, seed=seed)
    data, e = synth.quantize_half(v, kind)
    d_in = torch.from_numpy(np.ascontiguousarray(data.view(np.int16))).cuda().view(HALF_TORCH[dtype])
    return data, e, d_in, torch.from_numpy(np.ascontiguousarray(e)).cuda()


def _run(plan, fn, d_in, e_in, shape, inplace=False):
    nz, ny, nx = shape
    d_out = d_in.clone() if inplace else torch.full_like(d_in, float("nan"))
    src = d_out if inplace else d_in
    e_out = torch.full((ny, nx), 99, dtype=torch.int8, device="cuda")
    fn(plan, src, e_in, d_out, e_out)
    torch.cuda.synchronize()
    return d_out.view(torch.int16).cpu().numpy().view(np.uint16), e_out.cpu().numpy()


@pytest.mark.parametrize("direction", [FWD, BWD], ids=["fwd", "bwd"])
@pytest.mark.parametrize("dtype", [F16, BF16], ids=["f16", "bf16"])
@pytest.mark.parametrize("slabs", [1, 4])
def test_noalloc_equals_scaled_on_consecutive_calls(dtype, direction, slabs):
    # the second grid is smaller: it reuses the front of the static array
    # that the first call filled
    for i, shape in enumerate([(48, 40, 64), (24, 20, 32)]):
        nz, ny, nx = shape
        print(f"noalloc dtype {dtype} dir {direction} slabs {slabs} shape {shape}", flush=True)
        data, e, d_in, e_in = _inputs(shape, dtype, seed=100 + i)
        plan = croft.croft_plan_create_ex(nx, ny, nz, dtype, direction, 0, slabs)
        try:
            ref, ref_e = _run(plan, croft.croft_execute_scaled, d_in, e_in, shape)
            got, got_e = _run(plan, croft.croft_execute_scaled_noalloc, d_in, e_in, shape)
            got_ip, got_ip_e = _run(plan, croft.croft_execute_scaled_noalloc, d_in, e_in, shape, inplace=True)
        finally:
            croft.croft_plan_destroy(plan)
        assert np.array_equal(got, ref) and np.array_equal(got_e, ref_e), shape
        assert np.array_equal(got_ip, ref) and np.array_equal(got_ip_e, ref_e), shape
        kind = HALF_KIND[dtype]
        exact_in = oracle.decode_half(data, e, kind, 0)
        err = oracle.rel_l2(oracle.decode_half(got, got_e, kind, 2), oracle.dft3d(exact_in, direction))
        assert err <= TOL[dtype], (shape, err)


def test_noalloc_refuses_grids_beyond_the_static_array():
    # nx * nz = 4 MiB of exponents after the y pass, plus ny * nz before it
    nx, ny, nz = 2048, 2, 2048
    plan = croft.croft_plan_create(nx, ny, nz, F16, FWD)
    try:
        d = torch.zeros((nz, ny, nx, 2), dtype=torch.float16, device="cuda")
        e_out = torch.zeros((ny, nx), dtype=torch.int8, device="cuda")
        with pytest.raises(ValueError, match="static array holds 4194304"):
            croft.croft_execute_scaled_noalloc(plan, d, None, d, e_out)
        croft.croft_execute_scaled(plan, d, None, d, e_out)   # the plan's own scratch still serves it
        torch.cuda.synchronize()
        assert not e_out.any()
    finally:
        croft.croft_plan_destroy(plan)


def test_noalloc_refuses_other_dtypes_and_profiling():
    plan = croft.croft_plan_create(16, 16, 16, croft.CROFT_C64, FWD)
    d = torch.zeros((16, 16, 16), dtype=torch.complex64, device="cuda")
    e = torch.zeros((16, 16), dtype=torch.int8, device="cuda")
    try:
        with pytest.raises(ValueError, match="C16F"):
            croft.croft_execute_scaled_noalloc(plan, d, None, d, e)
    finally:
        croft.croft_plan_destroy(plan)
    plan = croft.croft_plan_create(16, 16, 16, F16, FWD)
    h = torch.zeros((16, 16, 16, 2), dtype=torch.float16, device="cuda")
    try:
        croft.croft_plan_profile(plan, True)
        with pytest.raises(ValueError, match="profiling"):
            croft.croft_execute_scaled_noalloc(plan, h, None, h, e)
        croft.croft_plan_profile(plan, False)
        croft.croft_execute_scaled_noalloc(plan, h, None, h, e)
        torch.cuda.synchronize()
    finally:
        croft.croft_plan_destroy(plan)
